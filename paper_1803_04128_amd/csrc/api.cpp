// C ABI entry points (include/bf.h): argument checks, plan construction,
// workspace, apply, query, destroy and error reporting.
#include <mutex>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "bf_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

// Runs an entry point's body with no C++ exception crossing the C ABI: a
// failed host allocation becomes BF_ENOMEM, anything else BF_EINVAL.
template <class F>
int guarded(const char* who, F&& body) {
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return fail(BF_ENOMEM, std::string(who) + ": host allocation failed");
    } catch (const std::exception& e) {
        return fail(BF_EINVAL, std::string(who) + ": " + e.what());
    } catch (...) {
        return fail(BF_EINVAL, std::string(who) + ": internal error");
    }
}

bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }

size_t env_bytes(const char* name, size_t dflt) {
    const char* s = std::getenv(name);
    if (!s || !*s) return dflt;
    char* end = nullptr;
    unsigned long long v = std::strtoull(s, &end, 10);
    return end && *end == 0 ? (size_t)v : dflt;
}

constexpr size_t kGiB = 1ull << 30;

}  // namespace

struct bf_plan_s {
    bfi::Plan p;
    unsigned magic = 0xbf00bf00u;
};

struct bf_graph_s {
    std::vector<bf_plan_s*> plans;   // each holds one graph reference
    hipGraphExec_t exec = nullptr;
    unsigned magic = 0xbf09bf09u;
};

namespace {

int path_of(const bfi::Plan& p) {
    if (!p.fused) return p.mfma ? BF_PATH_PER_STEP_MFMA : BF_PATH_PER_STEP;
    return p.mfma ? BF_PATH_FUSED : BF_PATH_FUSED_VALU;
}

void put_path(bfi::Plan& p, const bf_config& c) {
    p.fused = c.path == BF_PATH_FUSED || c.path == BF_PATH_FUSED_VALU;
    p.mfma = c.path == BF_PATH_FUSED || c.path == BF_PATH_PER_STEP_MFMA;
    p.tile_cols = c.tile_cols;
    p.switch_otf = c.switch_otf != 0;
    p.max_pass_levels = c.max_pass_levels;
    p.twiddle_otf = c.twiddle_otf != 0;
}

// Validates cfg against the plan and makes it current; the default workspace
// grows when the new form needs more.  On failure the plan is unchanged.
int apply_config(bfi::Plan& p, const bf_config& cfg) {
    if (cfg.path != BF_PATH_FUSED && cfg.path != BF_PATH_FUSED_VALU &&
        cfg.path != BF_PATH_PER_STEP && cfg.path != BF_PATH_PER_STEP_MFMA)
        return fail(BF_EINVAL, "bf_set_config: unknown path");
    if (cfg.tile_cols < 0 || cfg.tile_cols > 64 ||
        (cfg.tile_cols > 0 && cfg.tile_cols % p.r_amp != 0))
        return fail(BF_EINVAL,
                    "bf_set_config: tile_cols must be 0 or a multiple of r "
                    "up to 64");
    if (cfg.switch_otf != 0 && cfg.switch_otf != 1)
        return fail(BF_EINVAL, "bf_set_config: switch_otf must be 0 or 1");
    if (cfg.max_pass_levels < 0 || cfg.max_pass_levels > 12)
        return fail(BF_EINVAL, "bf_set_config: max_pass_levels must be 0..12");
    if (cfg.twiddle_otf != 0 && cfg.twiddle_otf != 1)
        return fail(BF_EINVAL, "bf_set_config: twiddle_otf must be 0 or 1");
    if (cfg.switch_otf && cfg.path != BF_PATH_PER_STEP_MFMA)
        return fail(BF_EUNSUPPORTED,
                    "bf_set_config: on-the-fly switch blocks exist in "
                    "BF_PATH_PER_STEP_MFMA only");
    const bool f0 = p.fused, m0 = p.mfma, o0 = p.switch_otf;
    const bool w0 = p.twiddle_otf;
    const int t0 = p.tile_cols, d0 = p.max_pass_levels;
    auto restore = [&] {
        p.fused = f0, p.mfma = m0, p.tile_cols = t0, p.switch_otf = o0;
        p.max_pass_levels = d0, p.twiddle_otf = w0;
    };
    put_path(p, cfg);
    std::string err = bfi::check_config(p);
    if (!err.empty()) {
        restore();
        return fail(BF_EUNSUPPORTED, "bf_set_config: " + err);
    }
    if (bfi::reads_stored_switch(p) && !p.S_arena) {
        if (hipDeviceSynchronize() != hipSuccess ||
            !bfi::build_switch_blocks(p).empty()) {
            (void)hipGetLastError();
            restore();
            return fail(BF_ENOMEM, "bf_set_config: switch block storage");
        }
    }
    const size_t need = bfi::workspace_bytes(p, p.max_nvec);
    if (need > p.ws_bytes) {
        void* nw = nullptr;
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMalloc(&nw, need) != hipSuccess) {
            (void)hipGetLastError();
            restore();
            return fail(BF_ENOMEM, "bf_set_config: workspace allocation");
        }
        (void)hipFree(p.ws);
        p.ws = nw;
        p.ws_bytes = need;
    }
    return BF_OK;
}

}  // namespace

extern "C" {

const char* bf_last_error(void) { return g_last_error.c_str(); }

int bf_points(int box_size, int q, int* out, int cap, int* count) {
    return guarded("bf_points", [&]() -> int {
        if (box_size < 1 || q < 2 || q > bfi::kMaxQ || !out || !count)
            return fail(BF_EINVAL, "bf_points: bad argument");
        int tmp[bfi::kMaxQ];
        int c = bfi::mock_chebyshev(box_size, q, tmp);
        if (c > cap) return fail(BF_EINVAL, "bf_points: capacity too small");
        std::memcpy(out, tmp, sizeof(int) * c);
        *count = c;
        return BF_OK;
    });
}

int bf_unwrap(const double* u, long long n, double tau, double* v,
              long long* disc, int cap, int* ndisc) {
    return guarded("bf_unwrap", [&]() -> int {
        if (!u || !v || !ndisc || n < 3 || !(tau > 0) || (cap > 0 && !disc) ||
            cap < 0)
            return fail(BF_EINVAL, "bf_unwrap: bad argument");
        return bfi::unwrap_vector(u, n, tau, v, disc, cap, ndisc);
    });
}

static bool sorted_unique(const long long* a, int n, long long N) {
    for (int i = 0; i < n; ++i) {
        if (a[i] < 0 || a[i] >= N) return false;
        if (i > 0 && a[i] <= a[i - 1]) return false;
    }
    return true;
}

int bf_recover_phase(long long N, const long long* C, int nc,
                     const long long* R, int nr, int rank, double tau,
                     bf_phase_sampler sample, void* ctx, int cap_rank,
                     double* U, double* V, int* rank_out) {
    return guarded("bf_recover_phase", [&]() -> int {
        if (N < 8 || !C || !R || nc < 1 || nr < 1 || rank < 1 || rank > 64 ||
            cap_rank < 1 || cap_rank > 64 || !(tau > 0) || !sample || !U ||
            !V || !rank_out)
            return fail(BF_EINVAL, "bf_recover_phase: bad argument");
        if (!sorted_unique(C, nc, N) || !sorted_unique(R, nr, N))
            return fail(BF_EINVAL,
                        "bf_recover_phase: C and R must be sorted, distinct and "
                        "in [0, N)");
        const int rc = bfi::recover_phase(N, C, nc, R, nr, rank, tau, sample,
                                          ctx, cap_rank, U, V, rank_out);
        if (rc != BF_OK)
            return fail(rc, std::string("bf_recover_phase: ") +
                                bfi::recovery_error());
        return BF_OK;
    });
}

int bf_lowrank_samples(long long N, const double* cols, const long long* C,
                       int nc, const double* rows, const long long* R, int nr,
                       int rank, int cap_rank, double* U, double* V,
                       int* rank_out) {
    return guarded("bf_lowrank_samples", [&]() -> int {
        if (N < 1 || !cols || !rows || !C || !R || nc < 1 || nr < 1 ||
            rank < 1 || rank > 64 || cap_rank < 1 || cap_rank > 64 || !U || !V ||
            !rank_out)
            return fail(BF_EINVAL, "bf_lowrank_samples: bad argument");
        if (!sorted_unique(C, nc, N) || !sorted_unique(R, nr, N))
            return fail(BF_EINVAL,
                        "bf_lowrank_samples: C and R must be sorted, distinct "
                        "and in [0, N)");
        const int rc = bfi::lowrank_fit(N, cols, C, nc, rows, R, nr, rank,
                                        cap_rank, U, V, rank_out);
        if (rc != BF_OK)
            return fail(rc, std::string("bf_lowrank_samples: ") +
                                bfi::recovery_error());
        return BF_OK;
    });
}

int bf_lagrange(const int* nodes, int r, const double* y, int m,
                double* out) {
    return guarded("bf_lagrange", [&]() -> int {
        if (!nodes || !y || !out || r < 1 || m < 0)
            return fail(BF_EINVAL, "bf_lagrange: bad argument");
        for (int i = 0; i < r; ++i)
            for (int j = i + 1; j < r; ++j)
                if (nodes[i] == nodes[j])
                    return fail(BF_EINVAL, "bf_lagrange: repeated node");
        bfi::lagrange_1d(nodes, r, y, m, out);
        return BF_OK;
    });
}

// Host part of plan construction: argument checks, trees, level schedule,
// execution form, vector chunking and the memory cap.  No device call.
static int configure_plan(const bf_grid* grid, const bf_phase* phase,
                          const bf_amplitude* amp, int q, int precision,
                          int max_nvec, int op, bfi::Plan& p) {
    if (!grid || !phase) return fail(BF_EINVAL, "bf_plan: NULL grid/phase");
    const int dim = grid->dim, n = grid->n;
    if (dim != 1 && dim != 2) return fail(BF_EINVAL, "bf_plan: dim must be 1 or 2");
    if (!is_pow2(n) || n < 2 || (dim == 1 && n > (1 << 22)) ||
        (dim == 2 && n > (1 << 11)))
        return fail(BF_EINVAL, "bf_plan: n must be a power of two in range");
    if (q < 2 || q > (dim == 1 ? bfi::kMaxQ : bfi::kMaxQ2D))
        return fail(BF_EINVAL, "bf_plan: q out of range");
    if (precision != BF_FP32 && precision != BF_BF16X3 &&
        precision != BF_FP16X3)
        return fail(BF_EINVAL, "bf_plan: unknown precision");
    if (max_nvec < 1) return fail(BF_EINVAL, "bf_plan: max_nvec < 1");
    if (op < BF_OP_N || op > BF_OP_H)
        return fail(BF_EINVAL, "bf_plan_op: unknown op");
    int need = -1;
    switch (phase->kind) {
        case BF_PHASE_DFT: need = 0; break;
        case BF_PHASE_FIO1D: need = dim == 1 ? 3 : -1; break;
        case BF_PHASE_RADON2D: need = dim == 2 ? 6 : -1; break;
        case BF_PHASE_SEPARABLE: need = 3; break;
        case BF_PHASE_FIO1D_WARP: need = dim == 1 ? 3 : -1; break;
        case BF_PHASE_LOWRANK: need = 0; break;
        default: return fail(BF_EINVAL, "bf_plan: unknown phase kind");
    }
    if (need < 0) return fail(BF_EINVAL, "bf_plan: phase kind needs another dim");
    if (phase->nparams != need || (need > 0 && !phase->params))
        return fail(BF_EINVAL, "bf_plan: wrong number of phase parameters");
    if (phase->kind == BF_PHASE_LOWRANK &&
        (phase->rank < 1 || phase->rank > 64 || !phase->U || !phase->V))
        return fail(BF_EINVAL,
                    "bf_plan: low-rank phase needs 1 <= rank <= 64, U and V");
    int r = 1;
    const double *a = nullptr, *b = nullptr;
    if (amp) {
        r = amp->r;
        a = amp->a;
        b = amp->b;
        if (r < 1 || r > bfi::kMaxAmp)
            return fail(BF_EINVAL, "bf_plan: amplitude rank out of range");
        if ((a == nullptr) != (b == nullptr))
            return fail(BF_EINVAL, "bf_plan: give both a and b or neither");
        if (!a && r != 1)
            return fail(BF_EINVAL, "bf_plan: alpha = 1 needs r = 1");
    }

    p.dim = dim;
    p.n = n;
    p.q = q;
    p.r_amp = r;
    p.precision = precision;
    p.max_nvec = max_nvec;
    p.has_amp = a != nullptr;
    p.phase.kind = phase->kind;
    p.phase.dim = dim;
    p.phase.n = n;
    p.phase.invn = 1.0 / (double)n;
    p.op = op;
    p.phase.transpose = (op & BF_OP_T) != 0;
    p.phase.conjugate = (op & BF_OP_C) != 0;
    for (int i = 0; i < need; ++i) p.phase.p[i] = phase->params[i];
    // initial execution form (bf_set_config / bf_autotune change it later)
    // default: fused passes in 1D, per-step MFMA launches in 2D (whose
    // 49- and 64-coefficient blocks the fused passes hold only on the
    // vector ALU)
    const char* fenv = std::getenv("BF_FUSED");
    p.fused = fenv ? std::atoi(fenv) != 0 : dim == 1;
    const char* menv = std::getenv("BF_MFMA");
    p.mfma = menv ? std::atoi(menv) != 0 : true;
    const char* tenv = std::getenv("BF_TILE_COLS");
    p.tile_cols = tenv ? std::max(0, std::atoi(tenv)) : 0;
    const char* oenv = std::getenv("BF_SWITCH_OTF");
    p.switch_otf = oenv && std::atoi(oenv) != 0 && !p.fused && p.mfma;
    // a plan built for the per-step MFMA form that evaluates its twiddles
    // in the apply stores none
    const char* wenv = std::getenv("BF_TWIDDLE_OTF");
    p.twiddle_otf = wenv && std::atoi(wenv) != 0 && !p.fused && p.mfma &&
                    precision == BF_FP32;
    p.tw_stored = !p.twiddle_otf;
    const char* senv = std::getenv("BF_SEP_SWITCH");
    p.sep_switch = !senv || std::atoi(senv) != 0;
    if (phase->kind == BF_PHASE_LOWRANK) p.phase.rank = phase->rank;
    std::string err = bfi::build_schedule(p);
    if (!err.empty()) return fail(BF_EUNSUPPORTED, "bf_plan: " + err);
    // memory: factors + workspace under the cap
    const size_t cap = env_bytes("BF_MEM_CAP_BYTES", (size_t)-1);
    const size_t ws_cap = env_bytes("BF_WS_CAP_BYTES", 16 * kGiB);
    size_t per_vec = 2 * (size_t)p.N * p.max_rank * p.r_amp * 8 + 64;
    int chunk = (int)std::max<size_t>(1, std::min<size_t>(max_nvec,
                                                         ws_cap / per_vec));
    p.chunk_nvec = chunk;
    size_t factor_est = (size_t)p.factor_stream_bytes +
                        (p.has_amp ? 2 * (size_t)r * p.N * 8 : 0) +
                        (phase->kind == BF_PHASE_LOWRANK
                             ? 2 * (size_t)phase->rank * p.N * 8
                             : 0);
    if (factor_est + per_vec * chunk > cap)
        return fail(BF_ENOMEM, "bf_plan: plan exceeds BF_MEM_CAP_BYTES");
    if (bfi::check_config(p) != "") {
        // the configured fused passes do not fit this plan
        if (precision != BF_FP32)
            return fail(BF_EUNSUPPORTED, "bf_plan: " + bfi::check_config(p));
        p.fused = false;
    }
    return BF_OK;
}

// Device bytes a configured plan allocates: factor arena, stored switch
// blocks (when its form reads them), low-rank phase factors, workspace.
static size_t plan_device_bytes(bfi::Plan& p) {
    return bfi::factor_arena_bytes(p) +
           (bfi::reads_stored_switch(p) ? bfi::switch_block_bytes(p) : 0) +
           (p.phase.kind == BF_PHASE_LOWRANK
                ? 2 * (size_t)p.phase.rank * p.N * sizeof(double)
                : 0) +
           bfi::workspace_bytes(p, p.max_nvec);
}

static int plan_impl(const bf_grid* grid, const bf_phase* phase,
                     const bf_amplitude* amp, int q, int precision,
                     int max_nvec, int op, bf_plan_t* out) {
    if (!out) return fail(BF_EINVAL, "bf_plan: out is NULL");
    *out = nullptr;
    bf_plan_s* h = new (std::nothrow) bf_plan_s();
    if (!h) return fail(BF_ENOMEM, "bf_plan: host allocation");
    bfi::Plan& p = h->p;
    if (int e = configure_plan(grid, phase, amp, q, precision, max_nvec, op,
                               p)) {
        delete h;
        return e;
    }
    const double* a = amp ? amp->a : nullptr;
    const double* b = amp ? amp->b : nullptr;
    std::string err;
    if (hipGetDevice(&p.device) != hipSuccess) {
        delete h;
        return fail(BF_EHIP, "bf_plan: no HIP device");
    }
    {
        // set-up of bf_apply_static's scratch on this device (a failure is
        // reported by bf_apply_static, which retries)
        void* unused = nullptr;
        (void)bfi::static_scratch(p.device, &unused);
        (void)hipGetLastError();
    }
    {
        // once per process: plans built on several host threads at once do
        // not race on the kernels' attribute flags (launches only read them)
        static std::once_flag attrs_once;
        std::call_once(attrs_once, [] { bfi::init_kernel_attrs(); });
    }
    if (phase->kind == BF_PHASE_LOWRANK) {
        const size_t fb = (size_t)p.N * phase->rank * sizeof(double);
        if (hipMalloc(&p.phase_arena, 2 * fb) != hipSuccess) {
            p.phase_arena = nullptr;
            err = "hipMalloc low-rank phase";
        } else {
            double* U = (double*)p.phase_arena;
            double* V = U + (size_t)p.N * phase->rank;
            if (hipMemcpy(U, phase->U, fb, hipMemcpyHostToDevice) !=
                    hipSuccess ||
                hipMemcpy(V, phase->V, fb, hipMemcpyHostToDevice) !=
                    hipSuccess)
                err = "hipMemcpy low-rank phase";
            p.phase.U = U;
            p.phase.V = V;
            p.phase.rank = phase->rank;
        }
    }
    if (err.empty()) err = bfi::build_factors(p);
    if (err.empty() && bfi::reads_stored_switch(p))
        err = bfi::build_switch_blocks(p);
    if (err.empty() && p.has_amp) err = bfi::upload_amplitude(p, a, b);
    if (err.empty()) {
        p.ws_bytes = bfi::workspace_bytes(p, max_nvec);
        if (hipMalloc(&p.ws, p.ws_bytes) != hipSuccess) {
            p.ws = nullptr;
            err = "workspace allocation failed";
        }
    }
    if (!err.empty()) {
        if (p.arena) (void)hipFree(p.arena);
        if (p.S_arena) (void)hipFree(p.S_arena);
        if (p.phase_arena) (void)hipFree(p.phase_arena);
        if (p.ws) (void)hipFree(p.ws);
        (void)hipGetLastError();
        delete h;
        return fail(err.find("alloc") != std::string::npos ||
                            err.find("Malloc") != std::string::npos
                        ? BF_ENOMEM
                        : BF_EHIP,
                    "bf_plan: " + err);
    }
    *out = h;
    return BF_OK;
}

int bf_lift_decide(long long N, int r1, const double* U1, const double* V1,
                   int r2, const double* U2, const double* V2, int r,
                   int r_eps, double eps, const double* omega, int omega_cols,
                   const long long* test_cols, int n_test, int rounds,
                   const long long* rows_s, const long long* cols_s,
                   int per_round, const long long* extra_rows,
                   const long long* extra_cols, int n_extra, int* y,
                   int* n_rank, double* P, double* Q, double* a, double* b,
                   int* k_out) {
    return guarded("bf_lift_decide", [&]() -> int {
        if (N < 4 || r1 < 1 || r2 < 1 || r < 1 || r >= r1 || r > 2 ||
            r_eps < 1 || !(eps > 0) || !U1 || !V1 || !U2 || !V2 || !omega ||
            omega_cols <= r1 || omega_cols > 64 || !test_cols || n_test < 1 ||
            rounds < 1 || per_round < 1 || !rows_s || !cols_s || n_extra < 0 ||
            (n_extra > 0 && (!extra_rows || !extra_cols)) || !y || !n_rank ||
            !P || !Q || !a || !b || !k_out || r_eps > 64 ||
            (long long)n_test > N || (long long)per_round > N)
            return fail(BF_EINVAL, "bf_lift_decide: bad argument");
        auto in_range = [&](const long long* v, long long n) {
            for (long long i = 0; i < n; ++i)
                if (v[i] < 0 || v[i] >= N) return false;
            return true;
        };
        if (!in_range(test_cols, n_test) ||
            !in_range(rows_s, (long long)rounds * per_round) ||
            !in_range(cols_s, (long long)rounds * per_round) ||
            !in_range(extra_rows, n_extra) || !in_range(extra_cols, n_extra))
            return fail(BF_EINVAL, "bf_lift_decide: index out of range");
        std::string err;
        int rc = bfi::lift_decide(N, r1, U1, V1, r2, U2, V2, r, r_eps, eps,
                                  omega, omega_cols, test_cols, n_test,
                                  rounds, rows_s, cols_s, per_round,
                                  extra_rows, extra_cols, n_extra, y, n_rank,
                                  P, Q, a, b, k_out, err);
        if (rc != BF_OK) return fail(rc, "bf_lift_decide: " + err);
        return BF_OK;
    });
}

int bf_plan_lifted(long long N, int r, const double* P, const double* Q,
                   int k, const double* a, const double* b, int max_nvec,
                   bf_plan_t* out) {
    return guarded("bf_plan_lifted", [&]() -> int {
        if (!out) return fail(BF_EINVAL, "bf_plan_lifted: out is NULL");
        *out = nullptr;
        if (N < 2 || N > (1LL << 24) || (r != 1 && r != 2) || k < 1 ||
            k > 64 || !P || !Q || !a || !b || max_nvec < 1)
            return fail(BF_EINVAL, "bf_plan_lifted: bad argument");
        for (long long i = 0; i < N * r; ++i)
            if (!std::isfinite(P[i]) || !std::isfinite(Q[i]))
                return fail(BF_EINVAL, "bf_plan_lifted: non-finite P or Q");
        bf_plan_s* h = new (std::nothrow) bf_plan_s();
        if (!h) return fail(BF_ENOMEM, "bf_plan_lifted: host allocation");
        bfi::Plan& p = h->p;
        p.dim = 1;
        p.n = (int)N;
        p.N = N;
        p.r_amp = k;
        p.max_nvec = max_nvec;
        p.fused = false;
        p.op = BF_OP_N;
        if (hipGetDevice(&p.device) != hipSuccess) {
            delete h;
            return fail(BF_EHIP, "bf_plan_lifted: no HIP device");
        }
        std::string err = bfi::nufft_build(p, r, P, Q, k, a, b);
        if (!err.empty()) {
            delete h;
            return fail(err.find("too large") != std::string::npos
                            ? BF_EUNSUPPORTED
                            : BF_EHIP,
                        "bf_plan_lifted: " + err);
        }
        const size_t ws_cap = env_bytes("BF_WS_CAP_BYTES", 16 * kGiB);
        const size_t per_vec = bfi::nufft_grid_bytes(*p.nufft, 1);
        p.chunk_nvec = (int)std::max<size_t>(
            1, std::min<size_t>(max_nvec, ws_cap / per_vec));
        p.ws_bytes = bfi::workspace_bytes(p, max_nvec);
        if (hipMalloc(&p.ws, p.ws_bytes) != hipSuccess) {
            p.ws = nullptr;
            bfi::nufft_free(p.nufft);
            delete h;
            return fail(BF_ENOMEM, "bf_plan_lifted: workspace allocation");
        }
        *out = h;
        return BF_OK;
    });
}

int bf_plan_footprint(const bf_grid* grid, const bf_phase* phase,
                      const bf_amplitude* amp, int q, int precision,
                      int max_nvec, int op, size_t* bytes) {
    return guarded("bf_plan_footprint", [&]() -> int {
        if (!bytes) return fail(BF_EINVAL, "bf_plan_footprint: NULL bytes");
        *bytes = 0;
        bfi::Plan p;
        if (int e = configure_plan(grid, phase, amp, q, precision, max_nvec,
                                   op, p))
            return e;
        *bytes = plan_device_bytes(p);
        return BF_OK;
    });
}

int bf_plan(const bf_grid* grid, const bf_phase* phase,
            const bf_amplitude* amp, int q, int precision, int max_nvec,
            bf_plan_t* out) {
    return guarded("bf_plan", [&]() -> int {
        return plan_impl(grid, phase, amp, q, precision, max_nvec, BF_OP_N, out);
    });
}

int bf_plan_op(const bf_grid* grid, const bf_phase* phase,
               const bf_amplitude* amp, int q, int precision, int max_nvec,
               int op, bf_plan_t* out) {
    return guarded("bf_plan_op", [&]() -> int {
        return plan_impl(grid, phase, amp, q, precision, max_nvec, op, out);
    });
}

static int check_plan(bf_plan_t plan) {
    if (!plan || plan->magic != 0xbf00bf00u)
        return fail(BF_EINVAL, "invalid plan handle");
    return BF_OK;
}

static int check_apply(bf_plan_t plan, int nvec, const void* f,
                       const void* g) {
    if (int e = check_plan(plan)) return e;
    const bfi::Plan& p = plan->p;
    if (nvec < 1 || nvec > p.max_nvec)
        return fail(BF_EINVAL, "bf_apply: nvec outside [1, max_nvec]");
    if (!f || !g) return fail(BF_EINVAL, "bf_apply: NULL f or g");
    const size_t bytes = (size_t)nvec * p.N * 8;
    const char* fb = (const char*)f;
    const char* gb = (const char*)g;
    if (fb < gb + bytes && gb < fb + bytes)
        return fail(BF_EINVAL, "bf_apply: f and g overlap");
    return BF_OK;
}

int bf_workspace_bytes(bf_plan_t plan, int nvec, size_t* bytes) {
    return guarded("bf_workspace_bytes", [&]() -> int {
        if (int e = check_plan(plan)) return e;
        if (!bytes || nvec < 1) return fail(BF_EINVAL, "bad argument");
        *bytes = bfi::workspace_bytes(plan->p, nvec);
        return BF_OK;
    });
}

int bf_apply_ws(bf_plan_t plan, int nvec, const void* f, void* g, void* ws,
                size_t ws_bytes, void* stream) {
    return guarded("bf_apply_ws", [&]() -> int {
        if (int e = check_apply(plan, nvec, f, g)) return e;
        if (!ws) return fail(BF_EINVAL, "bf_apply_ws: NULL workspace");
        bfi::Plan& p = plan->p;
        {
            const size_t vb = (size_t)nvec * p.N * 8;
            const char* w = (const char*)ws;
            const char* fb = (const char*)f;
            const char* gb = (const char*)g;
            if ((w < fb + vb && fb < w + ws_bytes) ||
                (w < gb + vb && gb < w + ws_bytes))
                return fail(BF_EINVAL, "bf_apply_ws: workspace overlaps f or g");
        }
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != p.device)
            return fail(BF_EINVAL, "bf_apply: plan belongs to another device");
        std::string err = bfi::launch_apply(p, nvec, f, g, ws, ws_bytes,
                                            (hipStream_t)stream);
        if (!err.empty()) return fail(BF_EHIP, "bf_apply: " + err);
        return BF_OK;
    });
}

int bf_apply_static(bf_plan_t plan, int nvec, const void* f, void* g,
                    void* stream) {
    return guarded("bf_apply_static", [&]() -> int {
        if (int e = check_apply(plan, nvec, f, g)) return e;
        bfi::Plan& p = plan->p;
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != p.device)
            return fail(BF_EINVAL,
                        "bf_apply_static: plan belongs to another device");
        const size_t need = bfi::workspace_bytes(p, 1);
        if (need > bfi::kStaticScratchBytes)
            return fail(BF_EINVAL,
                        "bf_apply_static: the plan needs " +
                            std::to_string(need) +
                            " bytes of workspace per vector, the static "
                            "scratch holds " +
                            std::to_string(bfi::kStaticScratchBytes));
        void* ws = nullptr;
        std::string err = bfi::static_scratch(p.device, &ws);
        if (!err.empty()) return fail(BF_EHIP, "bf_apply_static: " + err);
        err = bfi::launch_apply(p, nvec, f, g, ws, bfi::kStaticScratchBytes,
                                (hipStream_t)stream);
        if (!err.empty()) return fail(BF_EHIP, "bf_apply_static: " + err);
        return BF_OK;
    });
}

int bf_apply(bf_plan_t plan, int nvec, const void* f, void* g, void* stream) {
    return guarded("bf_apply", [&]() -> int {
        if (int e = check_plan(plan)) return e;
        return bf_apply_ws(plan, nvec, f, g, plan->p.ws, plan->p.ws_bytes, stream);
    });
}

static bool overlap(const void* a, const void* b, size_t bytes) {
    const char* ab = (const char*)a;
    const char* bb = (const char*)b;
    return ab < bb + bytes && bb < ab + bytes;
}

// Arguments of a chain (bf_apply_chain, bf_graph_create_chain).
static int check_chain(const char* who, const bf_plan_t* plans, int count,
                       int nvec, const void* f, const void* g,
                       const void* tmp) {
    if (!plans || count < 1) return fail(BF_EINVAL, std::string(who) + ": no plans");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess)
        return fail(BF_EHIP, std::string(who) + ": no HIP device");
    long long N = -1;
    for (int k = 0; k < count; ++k) {
        if (int e = check_apply(plans[k], nvec, f, g)) return e;
        const bfi::Plan& p = plans[k]->p;
        if (N >= 0 && p.N != N)
            return fail(BF_EINVAL, std::string(who) + ": plans differ in N");
        if (p.device != cur)
            return fail(BF_EINVAL, std::string(who) + ": plan on another device");
        N = p.N;
    }
    const size_t bytes = (size_t)nvec * N * 8;
    if (count > 1 && (!tmp || overlap(tmp, f, bytes) || overlap(tmp, g, bytes)))
        return fail(BF_EINVAL, std::string(who) + ": tmp NULL or overlapping");
    return BF_OK;
}

// The chain's applies on stream: apply k writes g when count - 1 - k is
// even, tmp otherwise, so the last one writes g and consecutive applies
// never read what they write.
static std::string launch_chain(const bf_plan_t* plans, int count, int nvec,
                                const void* f, void* g, void* tmp,
                                hipStream_t st) {
    const void* in = f;
    for (int k = 0; k < count; ++k) {
        void* out = ((count - 1 - k) % 2 == 0) ? g : tmp;
        bfi::Plan& p = plans[k]->p;
        std::string err = bfi::launch_apply(p, nvec, in, out, p.ws, p.ws_bytes, st);
        if (!err.empty()) return err;
        in = out;
    }
    return "";
}

int bf_apply_chain(const bf_plan_t* plans, int count, int nvec,
                   const void* f, void* g, void* tmp, void* stream) {
    return guarded("bf_apply_chain", [&]() -> int {
        if (int e = check_chain("bf_apply_chain", plans, count, nvec, f, g, tmp))
            return e;
        std::string err = launch_chain(plans, count, nvec, f, g, tmp,
                                       (hipStream_t)stream);
        if (!err.empty()) return fail(BF_EHIP, "bf_apply_chain: " + err);
        return BF_OK;
    });
}

int bf_destroy(bf_plan_t plan) {
    return guarded("bf_destroy", [&]() -> int {
        if (!plan) return BF_OK;
        if (int e = check_plan(plan)) return e;
        bfi::Plan& p = plan->p;
        if (p.graphs > 0)
            return fail(BF_EBUSY, "bf_destroy: captured graphs still use the plan");
        int rc = BF_OK;
        if (hipDeviceSynchronize() != hipSuccess) rc = BF_EHIP;
        if (p.arena && hipFree(p.arena) != hipSuccess) rc = BF_EHIP;
        if (p.S_arena && hipFree(p.S_arena) != hipSuccess) rc = BF_EHIP;
        if (p.phase_arena && hipFree(p.phase_arena) != hipSuccess) rc = BF_EHIP;
        if (p.ws && hipFree(p.ws) != hipSuccess) rc = BF_EHIP;
        bfi::nufft_free(p.nufft);
        p.nufft = nullptr;
        for (auto ev : p.prof.pool) (void)hipEventDestroy(ev);
        plan->magic = 0;
        delete plan;
        if (rc != BF_OK) return fail(rc, "bf_destroy: HIP error while freeing");
        return BF_OK;
    });
}

int bf_profile(bf_plan_t plan, int enable) {
    return guarded("bf_profile", [&]() -> int {
        if (int e = check_plan(plan)) return e;
        bfi::Profiler& pr = plan->p.prof;
        if (enable && pr.pool.empty()) {
            const int cap = 8192;
            pr.pool.resize(cap);
            for (int i = 0; i < cap; ++i) {
                if (hipEventCreate(&pr.pool[i]) != hipSuccess) {
                    for (int j = 0; j < i; ++j) (void)hipEventDestroy(pr.pool[j]);
                    pr.pool.clear();
                    return fail(BF_EHIP, "bf_profile: hipEventCreate failed");
                }
            }
        }
        pr.on = enable != 0;
        return BF_OK;
    });
}

int bf_profile_read(bf_plan_t plan, bf_kernel_stat* stats, int cap,
                    int* count) {
    return guarded("bf_profile_read", [&]() -> int {
        if (int e = check_plan(plan)) return e;
        if (!count || (cap > 0 && !stats))
            return fail(BF_EINVAL, "bf_profile_read: bad argument");
        bfi::Profiler& pr = plan->p.prof;
        std::vector<bf_kernel_stat> acc(pr.names.size());
        for (size_t i = 0; i < pr.names.size(); ++i) {
            std::memset(&acc[i], 0, sizeof(bf_kernel_stat));
            std::snprintf(acc[i].name, sizeof(acc[i].name), "%s",
                          pr.names[i].c_str());
        }
        for (const auto& r : pr.recs) {
            float ms = 0.f;
            if (hipEventSynchronize(pr.pool[r.ev1]) != hipSuccess ||
                hipEventElapsedTime(&ms, pr.pool[r.ev0], pr.pool[r.ev1]) !=
                    hipSuccess)
                return fail(BF_EHIP, "bf_profile_read: event query failed");
            bf_kernel_stat& k = acc[r.cls];
            k.launches += 1;
            k.total_ms += ms;
            k.bytes += r.bytes;
            k.flops += r.flops;
            k.state_bytes += r.state_bytes;
        }
        int n = 0;
        for (const auto& k : acc) {
            if (k.launches == 0) continue;
            if (n < cap) stats[n] = k;
            ++n;
        }
        *count = n;
        pr.recs.clear();
        pr.used = 0;
        return BF_OK;
    });
}

int bf_query(bf_plan_t plan, bf_plan_info* info) {
    return guarded("bf_query", [&]() -> int {
        if (int e = check_plan(plan)) return e;
        if (!info) return fail(BF_EINVAL, "bf_query: NULL info");
        const bfi::Plan& p = plan->p;
        std::memset(info, 0, sizeof(*info));
        info->dim = p.dim;
        info->n = p.n;
        info->L = p.L;
        info->h = p.h;
        info->q = p.q;
        info->r = p.r_amp;
        info->op = p.op;
        info->precision = p.precision;
        info->N = p.N;
        info->first_xi_level = p.l0;
        info->last_x_level = p.l1;
        info->n_steps = (int)p.steps.size();
        info->n_passes = p.fused ? bfi::fused_pass_count(p, p.chunk_nvec * p.r_amp)
                                 : (int)p.steps.size() + 1;
        info->max_rank = p.max_rank;
        info->chunk_nvec = p.chunk_nvec;
        info->factor_bytes = p.arena_bytes + p.S_bytes +
                             (p.phase_arena ? 2 * (size_t)p.phase.rank * p.N * 8
                                            : 0) +
                             (p.nufft ? bfi::nufft_factor_bytes(*p.nufft) : 0);
        info->method = p.nufft ? 1 : 0;
        info->workspace_bytes = p.ws_bytes;
        info->flops_per_column = p.flops_per_column;
        info->factor_stream_bytes = p.factor_stream_bytes;
        return BF_OK;
    });
}

int bf_step_query(bf_plan_t plan, int step, bf_step_info* info) {
    return guarded("bf_step_query", [&]() -> int {
        if (int e = check_plan(plan)) return e;
        const bfi::Plan& p = plan->p;
        if (!info || step < 0 || step >= (int)p.steps.size())
            return fail(BF_EINVAL, "bf_step_query: bad step or NULL info");
        const bfi::Step& s = p.steps[step];
        std::memset(info, 0, sizeof(*info));
        info->kind = s.kind;
        info->level = s.level;
        info->r_in = s.r_in;
        info->r_out = s.r_out;
        info->reads_f = s.reads_f ? 1 : 0;
        info->writes_lambda = s.writes_lambda ? 1 : 0;
        info->units = s.units;
        info->tw_entries = s.tw ? (long long)s.tw_elems : 0;
        info->S_entries = s.S ? (long long)s.S_elems : 0;
        info->side_in = s.ax_in.side;
        info->side_out = s.ax_out.side;
        return BF_OK;
    });
}

int bf_factor_entries(bf_plan_t plan, int step, int which,
                      const long long* idx, int count, long long* x,
                      long long* xi, float* values) {
    return guarded("bf_factor_entries", [&]() -> int {
        if (int e = check_plan(plan)) return e;
        const bfi::Plan& p = plan->p;
        if (step < 0 || step >= (int)p.steps.size() ||
            (which != 0 && which != 1) || count < 1 || !idx || !x || !xi ||
            !values)
            return fail(BF_EINVAL, "bf_factor_entries: bad argument");
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != p.device)
            return fail(BF_EINVAL,
                        "bf_factor_entries: plan belongs to another device");
        std::string err = bfi::read_factor_entries(p, step, which, idx,
                                                   count, x, xi, values);
        if (!err.empty())
            return fail(err.find("range") != std::string::npos ||
                                err.find("stores no") != std::string::npos
                            ? BF_EINVAL
                            : BF_EHIP,
                        "bf_factor_entries: " + err);
        return BF_OK;
    });
}

int bf_get_config(bf_plan_t plan, bf_config* cfg) {
    return guarded("bf_get_config", [&]() -> int {
        if (int e = check_plan(plan)) return e;
        if (!cfg) return fail(BF_EINVAL, "bf_get_config: NULL cfg");
        const bfi::Plan& p = plan->p;
        cfg->path = path_of(p);
        cfg->tile_cols = p.tile_cols;
        cfg->tile_cols_used =
            p.fused ? bfi::fused_tile_cols(p, p.chunk_nvec * p.r_amp) : 0;
        cfg->switch_otf = p.switch_otf ? 1 : 0;
        cfg->twiddle_otf = p.twiddle_otf ? 1 : 0;
        cfg->max_pass_levels = p.max_pass_levels;
        return BF_OK;
    });
}

int bf_set_config(bf_plan_t plan, const bf_config* cfg) {
    return guarded("bf_set_config", [&]() -> int {
        if (int e = check_plan(plan)) return e;
        if (!cfg) return fail(BF_EINVAL, "bf_set_config: NULL cfg");
        if (plan->p.nufft)
            return fail(BF_EUNSUPPORTED,
                        "bf_set_config: a NUFFT plan has one execution form");
        if (plan->p.graphs > 0)
            return fail(BF_EBUSY, "bf_set_config: captured graphs use the plan");
        return apply_config(plan->p, *cfg);
    });
}

int bf_autotune(bf_plan_t plan, int nvec, const void* f, void* g, int reps,
                void* stream, bf_tune_entry* out, int cap, int* count) {
    return guarded("bf_autotune", [&]() -> int {
        if (int e = check_apply(plan, nvec, f, g)) return e;
        if (plan->p.nufft)
            return fail(BF_EUNSUPPORTED,
                        "bf_autotune: a NUFFT plan has one execution form");
        if (reps < 1 || !count || (cap > 0 && !out))
            return fail(BF_EINVAL, "bf_autotune: bad argument");
        bfi::Plan& p = plan->p;
        if (p.graphs > 0)
            return fail(BF_EBUSY, "bf_autotune: captured graphs use the plan");
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != p.device)
            return fail(BF_EINVAL, "bf_autotune: plan belongs to another device");
        hipStream_t st = (hipStream_t)stream;
        // candidates: both fused forms at tile widths r * 2^j <= 16, the
        // MFMA passes also with each half split into two or three passes
        // (fusion depth), and the per-step launches; forms that resolve to
        // the same kernels are timed once
        int half = 0;
        {
            int nx = 0, nxi = 0;
            for (const auto& s : p.steps) {
                nxi += s.kind == bfi::STEP_XI;
                nx += s.kind == bfi::STEP_X;
            }
            half = std::max(nxi, nx);
        }
        std::vector<bf_config> cand;
        for (int path : {BF_PATH_FUSED, BF_PATH_FUSED_VALU})
            for (int tc = p.r_amp; tc <= 16; tc *= 2) {
                cand.push_back({path, tc, 0, 0, 0});
                if (path == BF_PATH_FUSED)
                    for (int parts = 2; parts <= 3; ++parts)
                        if (half >= 2 * parts)
                            cand.push_back({path, tc, 0, 0,
                                            (half + parts - 1) / parts});
            }
        cand.push_back({BF_PATH_PER_STEP, 0, 0, 0, 0});
        cand.push_back({BF_PATH_PER_STEP_MFMA, 0, 0, 0, 0});
        cand.push_back({BF_PATH_PER_STEP_MFMA, 0, 0, 1, 0});
        // the forms that evaluate the twiddles in the apply (the only ones
        // a plan built without stored twiddles runs)
        cand.push_back({BF_PATH_PER_STEP_MFMA, 0, 0, 0, 0, 1});
        cand.push_back({BF_PATH_PER_STEP_MFMA, 0, 0, 1, 0, 1});
        // the stored switch blocks are read by every candidate but two
        if (!p.S_arena && !bfi::build_switch_blocks(p).empty()) {
            (void)hipGetLastError();
            return fail(BF_ENOMEM, "bf_autotune: switch block storage");
        }
        const bool f0 = p.fused, m0 = p.mfma, o0 = p.switch_otf;
        const bool w0 = p.twiddle_otf;
        const int t0 = p.tile_cols, d0 = p.max_pass_levels;
        std::vector<bf_tune_entry> res;
        // (form, tile width, passes) timed
        std::vector<std::pair<int, int>> seen;
        size_t ws_need = 0;
        for (auto& c : cand) {
            put_path(p, c);
            bf_tune_entry e{};
            e.config = c;
            e.ms = -1.0;
            if (bfi::check_config(p).empty()) {
                e.config.tile_cols_used =
                    p.fused ? bfi::fused_tile_cols(p, std::min(nvec, p.chunk_nvec) *
                                                          p.r_amp)
                            : 0;
                // 2D plans (and r not a power of two) have no MFMA passes: the
                // fused form is then the vector-ALU one
                const bool mf = p.fused && p.mfma && p.dim == 1 &&
                                (p.r_amp & (p.r_amp - 1)) == 0 && p.r_amp <= 8;
                const int key =
                    !p.fused ? (p.mfma ? (p.switch_otf ? 4 : 3) +
                                             (p.twiddle_otf ? 2 : 0)
                                       : 2)
                             : (mf ? 0 : 1);
                const int np = p.fused ? bfi::fused_pass_count(
                                             p, std::min(nvec, p.chunk_nvec) *
                                                    p.r_amp)
                                       : 0;
                std::pair<int, int> k{key * 64 + np, e.config.tile_cols_used};
                bool dup = false;
                for (auto& s2 : seen) dup |= s2 == k;
                if (!dup) {
                    seen.push_back(k);
                    e.ms = 0.0;   // to be timed
                    ws_need = std::max(ws_need, bfi::workspace_bytes(p, nvec));
                } else {
                    e.ms = -2.0;
                }
            }
            res.push_back(e);
        }
        void* ws = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        std::string err;
        if (hipMalloc(&ws, std::max<size_t>(ws_need, 256)) != hipSuccess)
            err = "workspace allocation";
        if (err.empty() && (hipEventCreate(&e0) != hipSuccess ||
                            hipEventCreate(&e1) != hipSuccess))
            err = "event creation";
        const bool prof0 = p.prof.on;
        p.prof.on = false;
        int best = -1;
        for (size_t i = 0; i < res.size() && err.empty(); ++i) {
            if (res[i].ms != 0.0) continue;
            put_path(p, res[i].config);
            err = bfi::launch_apply(p, nvec, f, g, ws, ws_need, st);   // warm-up
            if (!err.empty()) break;
            if (hipEventRecord(e0, st) != hipSuccess) { err = "event record"; break; }
            for (int k = 0; k < reps && err.empty(); ++k)
                err = bfi::launch_apply(p, nvec, f, g, ws, ws_need, st);
            float ms = 0.f;
            if (err.empty() && (hipEventRecord(e1, st) != hipSuccess ||
                                hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                err = "event timing";
            if (!err.empty()) break;
            res[i].ms = ms / reps;
            if (best < 0 || res[i].ms < res[best].ms) best = (int)i;
        }
        p.prof.on = prof0;
        if (ws) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(ws);
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        p.fused = f0, p.mfma = m0, p.tile_cols = t0, p.switch_otf = o0;
        p.max_pass_levels = d0, p.twiddle_otf = w0;
        if (!err.empty()) {
            (void)hipGetLastError();
            return fail(BF_EHIP, "bf_autotune: " + err);
        }
        *count = (int)res.size();
        for (int i = 0; i < (int)res.size() && i < cap; ++i) out[i] = res[i];
        if (best < 0) return fail(BF_EUNSUPPORTED, "bf_autotune: no candidate ran");
        bf_config chosen = res[best].config;
        chosen.tile_cols_used = 0;
        return apply_config(p, chosen);
    });
}

// Captures the chain plans[0..count) (one plan: a plain apply) into an
// executable graph on a private stream.
static int capture_chain(const char* who, const bf_plan_t* plans, int count,
                         int nvec, const void* f, void* g, void* tmp,
                         bf_graph_t* out) {
    bf_graph_s* gr = new (std::nothrow) bf_graph_s();
    if (!gr) return fail(BF_ENOMEM, std::string(who) + ": host allocation");
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    std::string err;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        err = "stream creation";
    else if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) !=
             hipSuccess)
        err = "begin capture";
    else {
        for (int k = 0; k < count; ++k) plans[k]->p.capturing = true;
        std::string aerr = launch_chain(plans, count, nvec, f, g, tmp, cs);
        for (int k = 0; k < count; ++k) plans[k]->p.capturing = false;
        hipError_t ee = hipStreamEndCapture(cs, &graph);
        if (!aerr.empty()) err = aerr;
        else if (ee != hipSuccess || !graph) err = "end capture";
        else if (hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0) !=
                 hipSuccess)
            err = "graph instantiation";
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
    if (!err.empty()) {
        (void)hipGetLastError();
        delete gr;
        return fail(BF_EHIP, std::string(who) + ": " + err);
    }
    for (int k = 0; k < count; ++k) {
        gr->plans.push_back(plans[k]);
        ++plans[k]->p.graphs;
    }
    *out = gr;
    return BF_OK;
}

int bf_graph_create(bf_plan_t plan, int nvec, const void* f, void* g,
                    bf_graph_t* out) {
    return guarded("bf_graph_create", [&]() -> int {
        if (!out) return fail(BF_EINVAL, "bf_graph_create: out is NULL");
        *out = nullptr;
        if (int e = check_apply(plan, nvec, f, g)) return e;
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != plan->p.device)
            return fail(BF_EINVAL, "bf_graph_create: plan belongs to another device");
        return capture_chain("bf_graph_create", &plan, 1, nvec, f, g, nullptr,
                             out);
    });
}

int bf_graph_create_chain(const bf_plan_t* plans, int count, int nvec,
                          const void* f, void* g, void* tmp,
                          bf_graph_t* out) {
    return guarded("bf_graph_create_chain", [&]() -> int {
        if (!out) return fail(BF_EINVAL, "bf_graph_create_chain: out is NULL");
        *out = nullptr;
        if (int e = check_chain("bf_graph_create_chain", plans, count, nvec, f, g,
                                tmp))
            return e;
        return capture_chain("bf_graph_create_chain", plans, count, nvec, f, g,
                             tmp, out);
    });
}

int bf_graph_launch(bf_graph_t graph, void* stream) {
    return guarded("bf_graph_launch", [&]() -> int {
        if (!graph || graph->magic != 0xbf09bf09u)
            return fail(BF_EINVAL, "invalid graph handle");
        if (hipGraphLaunch(graph->exec, (hipStream_t)stream) != hipSuccess) {
            (void)hipGetLastError();
            return fail(BF_EHIP, "bf_graph_launch: hipGraphLaunch failed");
        }
        return BF_OK;
    });
}

int bf_graph_destroy(bf_graph_t graph) {
    return guarded("bf_graph_destroy", [&]() -> int {
        if (!graph) return BF_OK;
        if (graph->magic != 0xbf09bf09u)
            return fail(BF_EINVAL, "invalid graph handle");
        int rc = BF_OK;
        if (hipDeviceSynchronize() != hipSuccess) rc = BF_EHIP;
        if (hipGraphExecDestroy(graph->exec) != hipSuccess) rc = BF_EHIP;
        for (bf_plan_s* pl : graph->plans) --pl->p.graphs;
        graph->magic = 0;
        delete graph;
        if (rc != BF_OK) return fail(rc, "bf_graph_destroy: HIP error");
        return BF_OK;
    });
}

}  // extern "C"
