// Apply dispatch: vector chunking over the workspace and the choice between
// the per-step launches and the level-fused passes; the static scratch
// workspace of the allocation-free apply.
#include <algorithm>
#include <mutex>
#include <vector>

#include "apply_common.h"

namespace bfi {

// Workspace of bf_apply_static: a file-scope device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in symbol):
// it uses the device address hipGetSymbolAddress returns for the current
// device, recorded once per device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // device address per device ordinal
}  // namespace

std::string static_scratch(int device, void** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0) return "bad device";
    if ((size_t)device >= g_scratch_ptr.size())
        g_scratch_ptr.resize(device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != device)
            return "the scratch's device is not current";
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return std::string("hipGetSymbolAddress(scratch): ") +
                   hipGetErrorString(e);
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return "";
}

ProfScope::ProfScope(Plan& pl, hipStream_t s) : p(pl), st(s) {
    if (!p.prof.on || p.capturing ||
        p.prof.used + 2 > (int)p.prof.pool.size())
        return;
    ev0 = p.prof.used++;
    if (hipEventRecord(p.prof.pool[ev0], st) != hipSuccess) ev0 = -1;
}

void ProfScope::end(const std::string& name, double bytes, double flops,
                    double state_bytes) {
    if (ev0 < 0) return;
    const int ev1 = p.prof.used++;
    if (hipEventRecord(p.prof.pool[ev1], st) != hipSuccess) return;
    p.prof.recs.push_back(
        {p.prof.cls_of(name), ev0, ev1, bytes, flops, state_bytes});
}

std::string run_fused(Plan& p, int nv, const float2* f, float2* g,
                      float2* buf0, float2* buf1, hipStream_t st, bool dry);
size_t fused_state_bytes(const Plan& p, int Vs);

// Two ping-pong state buffers of N * max_rank * (nv * r) complex64 each
// (the fused passes pad the columns to whole tiles).
static size_t state_bytes(const Plan& p, int nv) {
    if (p.fused) return fused_state_bytes(p, nv * p.r_amp);
    return (size_t)p.N * p.max_rank * (size_t)nv * p.r_amp * sizeof(float2);
}

size_t workspace_bytes(const Plan& p, int nvec) {
    const int nv = std::min(nvec, p.chunk_nvec);
    if (p.nufft) return nufft_grid_bytes(*p.nufft, nv);
    return 2 * state_bytes(p, nv);
}

std::string launch_apply(Plan& p, int nvec, const void* fv, void* gv,
                         void* ws, size_t ws_bytes, hipStream_t st) {
    if (nvec < 1) return "no vectors";
    if (p.nufft)
        return launch_nufft(p, nvec, (const float2*)fv, (float2*)gv, ws,
                            ws_bytes, st);
    // vectors per chunk: as many as the workspace holds, at most chunk_nvec
    int chunk = std::min(nvec, p.chunk_nvec);
    while (chunk > 1 && 2 * state_bytes(p, chunk) > ws_bytes) --chunk;
    if (2 * state_bytes(p, chunk) > ws_bytes)
        return "workspace too small for one vector";
    {
        std::string why = split_form_error(p);
        if (!why.empty()) return why;
    }
    if (reads_stored_switch(p) && !p.S_arena) {
        for (const auto& s : p.steps)
            if (s.S_elems) return "switch blocks are not stored";
    }
    // as many chunks as that width needs, balanced: the first `extra` hold
    // base + 1 vectors, the rest base (no small tail chunk)
    const int nch = (nvec + chunk - 1) / chunk;
    const int base = nvec / nch, extra = nvec % nch;
    if (p.fused) {
        // every width this apply launches is planned before the first
        // launch, so a failure leaves g untouched
        const int widths[2] = {base + (extra ? 1 : 0), base};
        for (int nv : widths) {
            std::string err = run_fused(p, nv, nullptr, nullptr, nullptr,
                                        nullptr, nullptr, true);
            if (!err.empty()) return err;
        }
    }
    const float2* f = (const float2*)fv;
    float2* g = (float2*)gv;
    for (int c = 0, v0 = 0; c < nch; ++c) {
        const int nv = base + (c < extra ? 1 : 0);
        float2* b0 = (float2*)ws;
        float2* b1 = (float2*)((char*)ws + state_bytes(p, nv));
        std::string err =
            p.fused ? run_fused(p, nv, f + (size_t)v0 * p.N,
                                g + (size_t)v0 * p.N, b0, b1, st, false)
                    : run_basic(p, nv, f + (size_t)v0 * p.N,
                                g + (size_t)v0 * p.N, b0, b1, st);
        if (!err.empty()) return err;
        v0 += nv;
    }
    return "";
}

std::string split_form_error(const Plan& p) {
    if (p.precision == BF_FP32) return "";
    if (p.dim == 1 && !p.fused)
        return "split precision needs the fused passes in 1D";
    if (p.dim == 2 && (p.fused || !p.mfma || p.switch_otf))
        return "split precision needs the per-step MFMA form with stored "
               "switch blocks in 2D";
    return "";
}

std::string check_config(Plan& p) {
    if (p.nufft) return "";
    if (p.twiddle_otf && (p.fused || !p.mfma || p.precision != BF_FP32))
        return "twiddles are evaluated in the apply by the FP32 per-step "
               "MFMA form only";
    if (!p.tw_stored && !p.twiddle_otf)
        return "the plan stores no twiddles (built with BF_TWIDDLE_OTF): "
               "only the form that evaluates them runs it";
    {
        std::string why = split_form_error(p);
        if (!why.empty()) return why;
    }
    if (!p.fused) return "";
    // every chunk width the applies can take: the full chunk and a tail
    const int widths[2] = {p.chunk_nvec, 1};
    for (int nv : widths) {
        std::string err = run_fused(p, nv, nullptr, nullptr, nullptr, nullptr,
                                    nullptr, true);
        if (!err.empty()) return err;
    }
    return "";
}

}  // namespace bfi
