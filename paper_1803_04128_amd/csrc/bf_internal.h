// Internal plan structures of the butterfly library (host side).
//
// Notation follows Section 4 of the paper: trees T_X and T_Omega of depth L
// over an n^dim grid, tree level l, pairs (A, B) with A at level l of T_X and
// B at level L - l of T_Omega, switch level h = floor(L / 2) (L - floor(L / 2)
// when the plan factorizes the transposed kernel).  R = 2^dim is
// the number of children of a box.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bf.h"

namespace bfi {

constexpr int kMaxQ = 16;       // interpolation points per dimension (1D)
constexpr int kMaxQ2D = 8;      // per dimension in 2D
constexpr int kMaxRank = 64;    // coefficients per pair (8 x 8 in 2D)
constexpr int kMaxAmp = 16;     // amplitude rank

// Interpolation points of a box side, per dimension: `r1` 0-based offsets
// inside a side of `side` indices.  A box's points are the tensor product of
// these offsets over the dimensions, flattened row-major (t1 * r1 + t2).
struct Axis {
    int side;
    int r1;
    int off[kMaxQ];
};

enum StepKind { STEP_XI = 0, STEP_SWITCH = 1, STEP_X = 2 };

// One computed step of the regrouped Algorithm 4.1.
//
// STEP_XI (recursion in xi, eq. (eqn:2)) at level l: a unit (a', b), with a'
//   at level l-1 of T_X and b at level L-l of T_Omega, reads the R input
//   pairs (a', R b + c) and writes the R output pairs (R a' + i, b):
//     mu^{AB} = sum_c M_c (W_{A,C} . mu^{PC}),
//   M_c[t][s] = M_t^B(xi_s^C) (real, shared by all units), W the twiddle
//   exp(2 pi i [Phi(c_A, xi_s^C) - Phi(c_P, xi_s^C)]).  When the step reads
//   f directly (the exact levels below it are copies), W is
//   exp(2 pi i Phi(c_A, xi_s^C)).
// STEP_SWITCH at level h: per pair, nu^{AB} = S_{AB} mu^{AB}, S the residual
//   phase block exp(2 pi i [Phi(x_t^A, xi_s^B) - Phi(c_A, xi_s^B)
//   - Phi(x_t^A, c_B)]); the second term is absent when the switch reads f,
//   the third when no x step follows.
// STEP_X (recursion in x, eq. (eqn:3)) at level l: same unit shape,
//     nu^{AB} = sum_c T_{A,C} . (M_i nu^{PC}),
//   M_i[t][s] = M_s^P(x_t^A) for A the i-th child of P, T the twiddle
//   exp(2 pi i [Phi(x_t^A, c_C) - Phi(x_t^A, c_B)]); the last x step uses
//   exp(2 pi i Phi(x_t^A, c_C)) and so emits lambda for the final sums.
struct Step {
    int kind = 0;
    int level = 0;
    int r_in = 0, r_out = 0;
    bool reads_f = false;
    bool writes_lambda = false;
    Axis ax_in{}, ax_out{};
    long long units = 0;        // N / R for XI and X, N for the switch
    // device factors (inside the plan arena)
    float2* tw = nullptr;       // [units][R][R][r] (r = r_in for XI, r_out X)
    float* mats = nullptr;      // [R][r_out][r_in]
    float2* S = nullptr;        // [N][r_out][r_in]
    // split precisions (1D): hi and lo 16-bit parts of mats in the A-operand
    // order of the fused passes' 16x16x32 (xi: [lane][8], lane l holding
    // M_{e % 2}[l % 16][4 (l / 16) + e / 2]) or 16x16x16 products (x:
    // [child][lane][4], M_i[l % 16][4 (l / 16) + e]); zero past the ranks
    uint16_t* asplit_hi = nullptr;
    uint16_t* asplit_lo = nullptr;
    // mats in the A-operand order of a 16x16x4 FP32 MFMA, zero padded:
    // [R][ceil(r_out/16)][ceil(r_in/4)][lane], lane l holding
    // M[16 mt + l % 16][4 ks + l / 16]
    float* amat = nullptr;
    // 1D xi steps (r_out <= 16): [M_0 | M_1] as the A operand of a K = 2 r_in
    // product with the children interleaved, [ceil(r_in/2)][lane], lane l
    // holding M_{c}[l % 16][2 kk + (l / 16) / 2], c = (l / 16) % 2
    float* amat_xi = nullptr;
    size_t tw_elems = 0, mat_elems = 0, S_elems = 0, amat_elems = 0;
    size_t amat_xi_elems = 0;
    size_t asplit_elems = 0;  // 512 per step with a matrix (split plans)
    // split plans of the per-step form (2D): hi and lo 16-bit parts of mats
    // in the A order of 16x16x16 products, [R][ceil(r_out/16)][ceil(r_in/16)]
    // [lane][4], lane l holding M[16 mt + l % 16][16 kb + 4 (l / 16) + e]
    uint16_t* a16_hi = nullptr;
    uint16_t* a16_lo = nullptr;
    size_t a16_elems = 0;
    // 2D: the 1D factors L^0, L^1 of the Kronecker matrices ([2][b][a],
    // b = ax_out.r1, a = ax_in.r1) and their A tables for the
    // one-dimension-at-a-time contractions (apply_step_sep.hip): xi steps
    // [4][lane] = L^c[l % 16][s] at k = 4 ks + l / 16 = c a + s; x steps
    // [2][lane] = L^i[t][s] at row l % 16 = i b + t, s = 4 ks + l / 16
    std::vector<double> lag1_host;
    float* amat_sep = nullptr;
    size_t sep_elems = 0;
    std::vector<double> mats_host;  // FP64 Lagrange matrices
};

struct PhaseSpec {
    int kind;
    int dim;
    int n;
    int transpose;   // factorize K^T: phase roles of x and xi exchanged
    int conjugate;   // factorize the conjugate kernel: phase negated
    double invn;     // 1 / n (exact: n is a power of two)
    double p[6];
    // BF_PHASE_LOWRANK: device factors [N][rank] (Plan::phase_arena)
    const double* U;
    const double* V;
    int rank;
};

// A fused kernel pass: consecutive steps [first, last] executed by one
// launch per vector chunk.
struct Pass {
    int first, last;
    bool tail;        // ends with the final sums and the amplitude
    int group_log;    // log_R of pairs per group
};

// Timing records of kernel launches (bf_profile).
struct ProfRec {
    int cls;          // index into Profiler::names
    int ev0, ev1;     // indices into the event pool
    double bytes, flops, state_bytes;
};

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    int used = 0;
    std::vector<std::string> names;
    std::vector<ProfRec> recs;
    int cls_of(const std::string& n) {
        for (size_t i = 0; i < names.size(); ++i)
            if (names[i] == n) return (int)i;
        names.push_back(n);
        return (int)names.size() - 1;
    }
};

struct NufftPlan;   // nufft.hip

struct Plan {
    // a plan of the NUFFT path of Section 3 (eq. (eqn:tg3)) instead of the
    // butterfly: the fields below describe its grid (1D, N = n) only
    NufftPlan* nufft = nullptr;
    int dim = 1, n = 0, L = 0, h = 0, R = 2, q = 0, r_amp = 1;
    int precision = BF_FP32, max_nvec = 1;
    long long N = 0;
    PhaseSpec phase{};
    int l0 = 0, l1 = 0, lend = 0;
    int head_step_side = 1;   // side of the boxes the first step reads f over
    int tail_side = 1;        // side of the T_X boxes summed in the tail
    std::vector<Step> steps;
    int max_rank = 1;
    // device memory
    void* arena = nullptr;
    size_t arena_bytes = 0;
    void* S_arena = nullptr;  // stored switch blocks (build_switch_blocks)
    void* phase_arena = nullptr;  // low-rank phase factors on the device
    size_t S_bytes = 0;
    bool has_amp = false;     // false: alpha = 1 (r = 1)
    int op = 0;               // BF_OP_*: which of K, K^T, conj K, K^H
    // per-step MFMA form: generate the switch blocks during the apply
    // instead of reading the stored S
    bool switch_otf = false;
    // per-step MFMA form: evaluate the twiddles during the apply instead of
    // reading them; a plan built for that form (BF_TWIDDLE_OTF) stores none
    bool twiddle_otf = false;
    bool tw_stored = true;
    // 2D per-step MFMA form: the switch fused behind the last xi level
    // (BF_SEP_SWITCH=0 at plan time keeps them separate launches)
    bool sep_switch = true;
    float2* a_dev = nullptr;  // [r][N] complex64, nullptr when alpha = 1
    float2* b_dev = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int chunk_nvec = 1;
    int device = 0;
    bool fused = true;        // level-fused passes (else one launch per step)
    bool mfma = true;         // fused passes may use the MFMA kernels
    int tile_cols = 0;        // fused tile width override (0: heuristic)
    int max_pass_levels = 0;  // fused: levels per pass cap (0: LDS-bound)
    int graphs = 0;           // live captured graphs bound to ws
    bool capturing = false;   // inside a graph capture (no event records)
    double flops_per_column = 0;
    double factor_stream_bytes = 0;
    Profiler prof;
};

// Wraps a kernel launch with timing events when profiling is on.
struct ProfScope {
    Plan& p;
    hipStream_t st;
    int ev0 = -1;
    ProfScope(Plan& pl, hipStream_t s);
    // bytes: algorithmic bytes (inputs f, b, outputs g, a and factors,
    // each once); state_bytes: the state read or written between launches
    void end(const std::string& name, double bytes, double flops,
             double state_bytes = 0.0);
};

// geometry.cpp
int mock_chebyshev(int side, int q, int* off);
void lagrange_1d(const int* nodes, int r, const double* y, int m, double* out);
Axis make_axis(int side, int q);
std::string build_schedule(Plan& p);   // "" on success, else a message

// factors.hip
std::string build_factors(Plan& p);
std::string upload_amplitude(Plan& p, const double* a, const double* b);
std::string build_switch_blocks(Plan& p);
// device bytes build_factors / build_switch_blocks allocate (host only)
size_t factor_arena_bytes(Plan& p);
size_t switch_block_bytes(const Plan& p);
// diagnostic read-back of stored factor entries (which: 0 twiddles, 1 S)
std::string read_factor_entries(const Plan& p, int step, int which,
                                const long long* idx, int count,
                                long long* x_out, long long* xi_out,
                                float* val_out);
// phase recovery (recovery.cpp); arguments checked by the C ABI
int recover_phase(long long N, const long long* C, int nc, const long long* R,
                  int nr, int rank, double tau, bf_phase_sampler sample,
                  void* ctx, int cap_rank, double* U, double* V,
                  int* rank_out);
int unwrap_vector(const double* u, long long n, double tau, double* v,
                  long long* disc, int cap, int* ndisc);
int lowrank_fit(long long N, const double* cols, const long long* Cs, int mc,
                const double* rows, const long long* Rs, int mr, int rank,
                int cap_rank, double* U, double* V, int* rank_out);
const char* recovery_error();
// whether the plan's current execution form reads the stored switch blocks
inline bool reads_stored_switch(const Plan& p) {
    return !(p.switch_otf && !p.fused && p.mfma);
}
// bytes of the static scratch workspace of bf_apply_static (per device)
constexpr size_t kStaticScratchBytes = BF_STATIC_SCRATCH_BYTES;
// its device address on `device` (current), recorded on first use
std::string static_scratch(int device, void** out);
// apply_step_sep.hip: 2D per-step levels contracted per dimension
bool step_sep_ok(const Plan& p, const Step& s);
// the last xi level with the switch fused behind it (FP32, stored S)
bool sep_switch_ok(const Plan& p, const Step& xi, const Step& sw);
void init_step_sep_attrs();
// apply_step_split.hip: split-precision per-step kernels
void init_step_split_attrs();
// "" when the plan's execution form can run its precision
std::string split_form_error(const Plan& p);
// apply.hip
std::string launch_apply(Plan& p, int nvec, const void* f, void* g, void* ws,
                         size_t ws_bytes, hipStream_t stream);
size_t workspace_bytes(const Plan& p, int nvec);
std::string check_config(Plan& p);   // "" when every pass fits
// apply_fused.hip
int fused_tile_cols(const Plan& p, int Vs);
int fused_pass_count(const Plan& p, int Vs);
void init_kernel_attrs();

// Algorithmic flops of one computed step for Vc columns: per unit and
// column, the twiddle products (6 flops) and the real-matrix times complex
// contractions (4 flops per multiply-add) of the regrouped eqs. (eqn:2) and
// (eqn:3), the switch as a dense complex block (8 per multiply-add).  In 2D
// the shared matrices are Kronecker products of 1D ones (a inputs, b
// outputs per dimension), contracted one dimension at a time with the
// first stage shared: a xi output child sums its two second-dimension
// children before the first-dimension matrix (4 a^2 b + 2 a b^2 per child),
// an x input child forms its second-dimension products once for both
// first-dimension outputs (2 a^2 b + 4 a b^2 per child).
inline double step_alg_flops(int dim, int kind, long long units, int r_in,
                             int r_out, int a1, int b1, double Vc) {
    const int R = 1 << dim;
    const double U = (double)units * Vc;
    if (kind == STEP_SWITCH) return U * r_out * (double)r_in * 8.0;
    if (dim == 1) {
        if (kind == STEP_XI)
            return U * R * (R * r_in * 6.0 + (double)R * r_out * r_in * 4.0);
        return U * R * ((double)R * r_out * r_in * 4.0 + R * r_out * 8.0);
    }
    const double a = a1, b = b1;
    if (kind == STEP_XI)
        return U * (R * R * r_in * 6.0 + R * (4 * a * a * b + 2 * a * b * b) * 4.0);
    return U * (R * (2 * a * a * b + 4 * a * b * b) * 4.0 + R * R * r_out * 8.0);
}

inline double step_alg_flops(const Plan& p, const Step& s, double Vc) {
    return step_alg_flops(p.dim, s.kind, s.units, s.r_in, s.r_out,
                          s.ax_in.r1, s.ax_out.r1, Vc);
}

// nufft.hip: the NUFFT by dimension lifting (Section 3, eq. (eqn:tg3))
std::string nufft_build(Plan& p, int r, const double* P, const double* Q,
                        int K, const double* a, const double* b);
void nufft_free(NufftPlan* q);
size_t nufft_grid_bytes(const NufftPlan& q, int nv);
size_t nufft_factor_bytes(const NufftPlan& q);
std::string launch_nufft(Plan& p, int nvec, const float2* f, float2* g,
                         void* ws, size_t ws_bytes, hipStream_t st);
// lifting.cpp: Algorithm 6 with Algorithm 1 (host, FP64)
int lift_decide(long long N, int r1, const double* U1, const double* V1,
                int r2, const double* U2, const double* V2, int r, int r_eps,
                double eps, const double* omega, int omega_cols,
                const long long* test_cols, int n_test, int rounds,
                const long long* rows_s, const long long* cols_s,
                int per_round, const long long* extra_rows,
                const long long* extra_cols, int n_extra, int* y, int* n_rank,
                double* P, double* Q, double* a, double* b, int* k_out,
                std::string& err);

// tiny helpers
inline int ilog2(long long v) {
    int l = 0;
    while ((1LL << (l + 1)) <= v) ++l;
    return l;
}

}  // namespace bfi
