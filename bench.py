#!/usr/bin/env python3
"""Throughput of g = K f applies on one MI355X.

Workload (default): the largest single-GPU configuration, the 1D FIO at
N = 2^20, Phi = x xi + c(x)|xi| with c(x) = (2 + sin 2 pi x)/8, amplitude
alpha = 1 + 0.5 sin(2 pi x) cos(2 pi xi / N) as r = 4 separable terms,
q = 10 interpolation points, 256 complex64 Gaussian vectors applied in one
call (FP32; --precision for the split forms).  A step is one bf_apply of
all vectors with the inputs resident in HBM.

Prints one JSON line: N*nvec/s over the timed steps, p50/p99 per-apply
latency, the roofline of the dominant kernel (library-side HIP events over
the timed region; algorithmic bytes and flops of the method, the state
spilled between launches reported beside them), and the oracle timed on the
host on a bounded sample.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector / matrix (published)
BF16_PEAK_TFLOPS = 2500.0      # dense MFMA bf16 / fp16

WORKLOADS = {
    "fio1d_n262144_batched": dict(precision="fp32"),
    "fio1d_n1024": dict(precision="fp32"),
    "radon2d_n256": dict(precision="fp32"),
    "fio1d_n1048576_sweep": dict(precision="fp32"),
}


# host-only sources that neither generate nor launch kernels: the C ABI
# layer and the phase recovery
HOST_ONLY = ("api.cpp", "recovery.cpp", "lifting.cpp")


def kernel_source_hash():
    """Hash of the sources that define the kernels and how they are launched
    (every csrc file but the host-only ones); a traffic record is valid for
    the kernels it was measured on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1803_04128_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name in HOST_ONLY:
            continue
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload, precision, kernel):
    """HBM bytes per launch measured with rocprofv3 counters, if recorded for
    the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    key = f"{workload}/{precision}/{kernel}"
    ent = rec.get(key)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def host_cpu():
    """(logical CPUs this process may use, CPU model) of the host."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return n, model


# amplitude columns (N * r) up to which the whole first vector is timed; a
# larger workload times one amplitude column (about 10-30 s of host work)
FULL_VECTOR_COLUMNS = 1 << 20


def cpu_baseline(w, f64, ab, g_gpu, phase=None, op="N"):
    """The oracle's FP64 butterfly timed on the host on a bounded sample of
    the workload: the first vector with all r amplitude columns when N r is
    at most 2^20 (then also the error of the GPU result for that vector),
    else the single column b_1 * f_0 of the full-N transform, scaled to
    N·nvec/s by the r columns a vector needs.  phase: (kind, params)
    replacing the workload's; op: the operator the plan applies.  Returns
    (report, rel err or None)."""
    import numpy as np
    from oracle.butterfly import butterfly_apply, butterfly_matvec
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] +
                    [1])
    except Exception:
        cores = 1
    nproc, model = host_cpu()
    kind, params = phase or (w.phase_kind, w.phase_params)
    flags = dict(transpose=op in ("T", "H"), conjugate=op in ("C", "H"))
    full = w.N * w.r <= FULL_VECTOR_COLUMNS
    err = None
    t0 = time.perf_counter()
    if ab is None:
        ref = butterfly_apply(w.dim, w.n, kind, params, w.q, f64[:1], **flags)
    elif full:
        ref = butterfly_matvec(w.dim, w.n, kind, params, w.q, ab[0], ab[1],
                               f64[:1], **flags)
    else:
        # one amplitude column: the butterfly of b_1 * f_0 (the recombination
        # with a_1 is O(N) and not timed)
        col = (ab[0] if op in ("T", "H") else ab[1])[0] * f64[0]
        butterfly_apply(w.dim, w.n, kind, params, w.q, col[None, :], **flags)
    dt = time.perf_counter() - t0
    cols = 1 if (ab is None or full) else w.r
    if ab is None or full:
        err = float(np.linalg.norm(g_gpu[0] - ref[0]) /
                    np.linalg.norm(ref[0]))
        what = (f"1 of {w.nvec} vectors x {w.r} amplitude terms, full "
                f"N={w.N}")
    else:
        what = (f"1 amplitude column (b_1 f_0) of {w.r} x {w.nvec} vectors, "
                f"full N={w.N}, rate scaled by the {w.r} columns a vector "
                f"needs")
    rep = {"value": w.N / (dt * cols), "unit": "N·nvec/s",
           "cores": int(cores), "nproc": nproc, "cpu_model": model,
           "kind": "oracle",
           "sample": f"FP64 step-by-step butterfly (NumPy), {what}; "
                     f"{dt:.1f} s"}
    return rep, err


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fio1d_n1048576_sweep",
                    choices=sorted(WORKLOADS) + ["serving", "composition",
                                                 "lifted"],
                    help="'serving': the continuous-batching server on the "
                         "mixed request stream; 'composition': the chained "
                         "applies L(L f) (each its own JSON line); "
                         "'lifted': NUFFT by dimension lifting against the "
                         "butterfly on one kernel")
    ap.add_argument("--requests", type=int, default=2000,
                    help="serving: requests per load level")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of the apply captured in a HIP graph "
                         "(bf_graph_create / bf_graph_launch)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the execution forms first and keep the "
                         "fastest (bf_autotune)")
    ap.add_argument("--switch-otf", action="store_true",
                    help="per-step MFMA form with the switch blocks "
                         "generated during the apply")
    ap.add_argument("--twiddle-otf", action="store_true",
                    help="per-step MFMA form with the twiddles evaluated "
                         "during the apply (the plan stores none; with "
                         "--switch-otf no factor is stored)")
    ap.add_argument("--op", default="N", choices=["N", "T", "C", "H"],
                    help="operator: K, K^T, conj(K) or K^H (bf_plan_op)")
    ap.add_argument("--lowrank-phase", type=int, default=0, metavar="RANK",
                    help="replace the workload's phase by a seeded phase "
                         "given as real low-rank factors of this rank")
    ap.add_argument("--comp-n", type=int, default=None,
                    help="composition and lifted: grid size N (a power of "
                         "two; defaults 2^18 and 2^16)")
    ap.add_argument("--precision", default=None,
                    choices=["fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--nvec", type=int, default=None,
                    help="override the workload's vector count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy before the timed "
                         "region (reference for hardware byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU "
              "path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "serving":
        serve_bench(args)
        return
    if args.workload == "composition":
        args.comp_n = args.comp_n or 1 << 18
        composition_bench(args)
        return
    if args.workload == "lifted":
        args.comp_n = args.comp_n or 1 << 16
        lifted_bench(args)
        return

    import numpy as np
    import torch

    import paper_1803_04128_amd as bfm
    from synthetic import CONFIGS, gaussian_vectors, amplitude_factors

    w = CONFIGS[args.workload]
    precision = args.precision or WORKLOADS[args.workload]["precision"]
    nvec = args.nvec or w.nvec
    f64 = gaussian_vectors(w.N, nvec, w.seed)
    f32 = f64.astype(np.complex64)
    ab = None
    if w.amplitude != "one":
        ab = amplitude_factors(w.amplitude, w.dim, w.n, w.r, w.amp_seed)
        ab = tuple(x.astype(np.complex64).astype(np.complex128) for x in ab)

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    f = torch.from_numpy(f32).to(dev)
    g = torch.empty_like(f)
    # the library's one-time set-up (code object load, kernel attributes)
    # happens at the first plan of the process: take it on a small plan so
    # that plan_s times this plan's construction alone
    bfm.Plan(1, 64, "dft", (), q=8).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.switch_otf:
        # read at plan construction: the plan then stores no switch blocks
        os.environ["BF_FUSED"] = "0"
        os.environ["BF_SWITCH_OTF"] = "1"
    if args.twiddle_otf:
        # read at plan construction: the plan then stores no twiddles
        os.environ["BF_FUSED"] = "0"
        os.environ["BF_TWIDDLE_OTF"] = "1"
    phase = (w.phase_kind, w.phase_params)
    if args.lowrank_phase:
        from synthetic import lowrank_phase
        phase = ("lowrank", lowrank_phase(w.dim, w.n, args.lowrank_phase, 21))
    plan = bfm.Plan(w.dim, w.n, phase[0], phase[1], q=w.q, amplitude=ab,
                    precision=precision, max_nvec=nvec, op=args.op)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan.info()

    if args.switch_otf or args.twiddle_otf:
        plan.set_config("per_step_mfma", switch_otf=args.switch_otf,
                        twiddle_otf=args.twiddle_otf)
    tune = None
    if args.autotune:
        tune = plan.autotune(f, out=g, reps=2)
    graph = plan.graph(f, g) if args.graph else None

    def step(stream):
        if graph is not None:
            graph.launch(stream=stream)
        else:
            plan.apply(f, out=g, stream=stream)

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    plan.profile(True)
    plan.profile_read()                      # clear
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        step(stream)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.profile(False)
    kstats = plan.profile_read()
    if graph is not None:
        # graph replays carry no library events: per-kernel times (for the
        # roofline) come from eager applies after the timed region
        plan.profile(True)
        for _ in range(max(3, min(args.steps, 20))):
            plan.apply(f, out=g, stream=stream)
        plan.profile(False)
        kstats = plan.profile_read()
    lat = np.array([evs[k].elapsed_time(evs[k + 1])
                    for k in range(args.steps)])

    value = w.N * nvec * args.steps / elapsed
    ms_per_step = elapsed * 1e3 / args.steps

    # dominant kernel: largest total time over the timed region
    name, st = max(kstats.items(), key=lambda kv: kv[1]["total_ms"])
    per_launch_ms = st["total_ms"] / st["launches"]
    ai = st["flops"] / max(st["bytes"], 1.0)
    if precision == "fp32":
        peak_c, unit_c = FP32_PEAK_TFLOPS, "TFLOP/s"
    else:
        peak_c, unit_c = BF16_PEAK_TFLOPS, "TFLOP/s"
    ridge = peak_c * 1e12 / (HBM_PEAK_GBS * 1e9)
    # the counters were taken on the workload's default form and batch
    default_form = not (args.switch_otf or args.twiddle_otf or args.autotune
                        or args.graph or args.op != "N" or args.lowrank_phase
                        or args.nvec)
    traffic = (traffic_from_profiles(args.workload, precision, name)
               if default_form else None)
    if ai >= ridge:
        achieved = st["flops"] / (st["total_ms"] * 1e-3) / 1e12
        # the vector-ALU forms are the *_basic steps and the plain passes;
        # every other kernel contracts on MFMA
        valu = name.endswith("_basic") or name in ("xi_pass", "x_pass")
        roof = {"bound": "alu" if valu else "mfma",
                "achieved": achieved, "peak": peak_c, "unit": unit_c,
                "frac": achieved / peak_c, "traffic": traffic}
    else:
        achieved = st["bytes"] / (st["total_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic}
    roof.update({"kernel": name, "launch_ms": per_launch_ms,
                 "alg_bytes_per_launch": st["bytes"] / st["launches"],
                 "alg_flops_per_launch": st["flops"] / st["launches"],
                 "state_bytes_per_launch": st["state_bytes"] /
                 st["launches"]})

    out = {
        "metric": "Kf applies: N·nvec/s",
        "value": value,
        "unit": "N·nvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x3": "bf16x3+f32",
                  "fp16x3": "f16x3+f32"}[precision],
        "data": "synthetic",
        "config": {"workload": w.name, "dim": w.dim, "N": w.N, "nvec": nvec,
                   "r": w.r, "q": w.q,
                   "phase": (f"lowrank(rank {args.lowrank_phase})"
                             if args.lowrank_phase else w.phase),
                   "op": args.op, "precision": precision},
        "latency_ms": {"p50": float(np.percentile(lat, 50)),
                       "p99": float(np.percentile(lat, 99))},
        "plan_s": plan_s,
        "kernels": {k: {"launches": v["launches"],
                        "ms_per_launch": v["total_ms"] / v["launches"],
                        "alg_flops_per_launch": v["flops"] / v["launches"],
                        "alg_bytes_per_launch": v["bytes"] / v["launches"],
                        "state_bytes_per_launch": v["state_bytes"] /
                        v["launches"]}
                    for k, v in kstats.items()},
        "apply_roofline_frac": (sum(v["flops"] for v in kstats.values()) /
                                elapsed / 1e12 /
                                peak_c),
        "roofline": roof,
        "exec": dict(plan.config(), graph=graph is not None),
        "factor_bytes": info["factor_bytes"],
    }
    if tune is not None:
        out["autotune"] = tune
    if not args.no_cpu_baseline:
        g_host = g[:1].cpu().numpy().astype(np.complex128)
        rep, err = cpu_baseline(w, f64.astype(np.complex64).astype(
            np.complex128), ab, g_host, phase=phase, op=args.op)
        out["cpu_baseline"] = rep
        if err is not None:
            out["rel_err_vs_oracle"] = err
    if graph is not None:
        graph.close()
    plan.close()
    print(json.dumps(out), flush=True)


def lifted_bench(args):
    """Section 3's choice between NUFFT and butterfly on one kernel: the
    wave-equation-like phase Phi = x xi + tau c(x)|xi| (tau = 8/N, c(x) =
    (2 + sin 2 pi x)/8) given as real rank-2 factors, alpha = 1, N = 2^16
    (--comp-n) and 16 vectors by default.  Algorithm 6 runs on the host
    (bf_lift_decide: r = 1, r_eps = 24, q = 3, eps = 1e-9, seeded draws);
    the lifted plan (eq. (eqn:tg3), bf_plan_lifted) and the butterfly plan
    of the same low-rank phase (q = 10) are timed on the same vectors.
    value: the lifted apply's N·nvec/s, the butterfly's beside it; the
    cpu_baseline leg times the dense FP64 rows (oracle) on 64 seeded rows and
    reports both GPU results' errors there."""
    import numpy as np
    import torch

    import paper_1803_04128_amd as bfm
    from synthetic import gaussian_vectors, sample_rows

    N = args.comp_n
    nvec = args.nvec or 16
    r_eps, q_os, eps, q_bf = 24, 3, 1e-9, 10
    x = np.arange(N) / N
    xi = (np.arange(N) - N // 2).astype(float)
    c = (2 + np.sin(2 * np.pi * x)) / 8
    U1 = np.stack([x, (8.0 / N) * c], 1)
    V1 = np.stack([xi, np.abs(xi)], 1)
    ones = np.ones((N, 1))
    rng = np.random.default_rng(12)
    omega = rng.standard_normal((N, 5))
    test = rng.choice(N, r_eps * q_os, replace=False)
    rows_s = np.stack([rng.choice(N, r_eps * q_os, replace=False)
                       for _ in range(2)])
    cols_s = np.stack([rng.choice(N, r_eps * q_os, replace=False)
                       for _ in range(2)])
    extra = (rng.choice(N, 4, replace=False), rng.choice(N, 4, replace=False))
    t0 = time.perf_counter()
    y, n_rank, P, Q, a, b = bfm.lift_decide(U1, V1, ones, ones, 1, r_eps, eps,
                                            omega, test,
                                            (rows_s, cols_s) + extra)
    decide_s = time.perf_counter() - t0
    if y != 1:
        print(json.dumps({"error": "Algorithm 6 refused the kernel",
                          "n_rank": int(n_rank)}), flush=True)
        sys.exit(1)
    f64 = gaussian_vectors(N, nvec, 3)
    f = torch.from_numpy(f64.astype(np.complex64)).to("cuda")
    t0 = time.perf_counter()
    lifted = bfm.plan_lifted(P, Q, a, b, max_nvec=nvec)
    torch.cuda.synchronize()
    lifted_plan_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    bf = bfm.Plan(1, N, "lowrank", (U1, V1), q=q_bf, max_nvec=nvec)
    torch.cuda.synchronize()
    bf_plan_s = time.perf_counter() - t0

    def timed(pl):
        g = torch.empty_like(f)
        for _ in range(args.warmup):
            pl.apply(f, out=g)
        torch.cuda.synchronize()
        pl.profile(True)
        pl.profile_read()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            pl.apply(f, out=g)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        pl.profile(False)
        kern = {k: {"launches": v["launches"],
                    "ms_per_launch": v["total_ms"] / v["launches"]}
                for k, v in pl.profile_read().items()}
        return el, kern, g.cpu().numpy().astype(np.complex128)

    el_l, kern_l, g_l = timed(lifted)
    el_b, kern_b, g_b = timed(bf)
    lifted.close()
    bf.close()
    out = {"metric": "Kf applies: N·nvec/s",
           "value": N * nvec * args.steps / el_l, "unit": "N·nvec/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": el_l * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "lifted1d_wave", "N": N, "nvec": nvec,
                      "r": 1, "r_eps": r_eps, "q_bf": q_bf},
           "decision": {"y": int(y), "sampled_rank": int(n_rank),
                        "terms": int(a.shape[0]), "host_s": decide_s},
           "plan_s": {"lifted": lifted_plan_s, "butterfly": bf_plan_s},
           "butterfly": {"value": N * nvec * args.steps / el_b,
                         "ms_per_step": el_b * 1e3 / args.steps,
                         "kernels": kern_b},
           "kernels": kern_l}
    if not args.no_cpu_baseline:
        from oracle.dense import dense_rows
        rows = sample_rows(N, 64, 5)
        nproc, model = host_cpu()
        t0 = time.perf_counter()
        ref = dense_rows(1, N, "lowrank", (U1, V1), "one", f64, rows)
        dt = time.perf_counter() - t0

        def err(g):
            return float(np.max(np.linalg.norm(g[:, rows] - ref, axis=1) /
                                np.linalg.norm(ref, axis=1)))
        out["cpu_baseline"] = {
            "value": rows.size * nvec / dt, "unit": "N·nvec/s", "cores": 1,
            "nproc": nproc, "cpu_model": model, "kind": "oracle",
            "sample": f"dense FP64 rows of K (NumPy), 64 seeded rows x "
                      f"{nvec} vectors; {dt:.1f} s"}
        out["rel_err_vs_dense"] = {"lifted": err(g_l), "butterfly": err(g_b)}
    print(json.dumps(out), flush=True)


def composition_bench(args):
    """L(L f) of the composition example (eq. (eq:example4), phase of eq.
    (eqn:FIOK2)), by default at the batched benchmark's size (N = 2^18, 64
    vectors, q = 10), as the chain [L, F, L] (bf_apply_chain, or one
    captured graph with --graph), F the Fourier-coefficient plan.  One JSON
    line with the chain's throughput and per-kernel times (eager applies)."""
    import numpy as np
    import torch

    import paper_1803_04128_amd as bfm
    from synthetic import PHASE_PARAMS, gaussian_vectors

    n, nvec, q = args.comp_n, args.nvec or 64, 10
    f = torch.from_numpy(gaussian_vectors(n, nvec, 1).astype(
        np.complex64)).to("cuda")
    g = torch.empty_like(f)
    tmp = torch.empty_like(f)
    t0 = time.perf_counter()
    L = bfm.Plan(1, n, "fio1d_warp", PHASE_PARAMS["fio1d_warp"], q=q,
                 max_nvec=nvec)
    F = bfm.fourier_coefficients_plan(n, q, max_nvec=nvec)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    graph = bfm.graph_chain([L, F, L], f, g, tmp) if args.graph else None

    def step():
        if graph is not None:
            graph.launch()
        else:
            bfm.apply_chain([L, F, L], f, out=g, tmp=tmp)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for pl in (L, F):
        pl.profile(True)
        pl.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if graph is not None:
        graph.close()
    kern = {}
    for tag, pl in (("L", L), ("F", F)):
        pl.profile(False)
        for k, v in pl.profile_read().items():
            kern[f"{tag}:{k}"] = {"launches": v["launches"],
                                  "ms_per_launch": v["total_ms"] /
                                  v["launches"]}
    out = {"metric": "L(L f) applies: N·nvec/s",
           "value": n * nvec * args.steps / elapsed, "unit": "N·nvec/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": elapsed * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "fio1d_warp_composition", "N": n,
                      "nvec": nvec, "q": q, "chain": "L, F, L",
                      "graph": graph is not None},
           "plan_s": plan_s, "kernels": kern}
    L.close()
    F.close()
    print(json.dumps(out), flush=True)


def serve_bench(args):
    """Serving: 39 resident plans (1D FIO at every N = 2^12..2^20, odd and
    even depths, and 2D Radon n = 64..512, each with amplitude rank r = 1,
    2 or 4), a seeded request mix with 1..32 vectors per request.  First every request arrives at once (saturation throughput),
    then Poisson arrivals at 0.5x, 0.8x and 1.2x that request rate; each
    level reports p50/p99 latency from arrival to completion on the GPU."""
    import numpy as np
    import torch

    from paper_1803_04128_amd.serving import (PlanSpec, Request, Server,
                                              overlap_fraction, summarize)
    from synthetic import (PHASE_PARAMS, SERVING_SHAPES, amplitude_factors,
                           gaussian_vectors, serving_requests)

    max_batch = 32
    # every plan of the mix resident at once (about 143 GiB of factors,
    # workspaces and staging for 32-vector batches) within the 288 GB of HBM
    srv = Server(hbm_budget_bytes=200 << 30, max_batch=max_batch)
    pools, Ns = [], {}
    for i, ((dim, n, phase, amp, r, q), _) in enumerate(SERVING_SHAPES):
        ab = None
        if amp != "one":
            ab = amplitude_factors(amp, dim, n, r, 11)
        name = f"s{i}"
        srv.register(name, PlanSpec(dim, n, phase, PHASE_PARAMS[phase], q=q,
                                    amplitude=ab))
        Ns[name] = n ** dim
        f = torch.from_numpy(gaussian_vectors(n ** dim, max_batch, 40 + i)
                             .astype(np.complex64)).to("cuda")
        pools.append((f, torch.empty_like(f)))
    # plans are resident before the clock starts (built once, reused)
    t0 = time.perf_counter()
    for i in range(len(SERVING_SHAPES)):
        rp = srv.cache.get(f"s{i}")
        rp.plan.apply(pools[i][0], out=pools[i][1])
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0

    def stream(rate, seed):
        out = []
        for k, (t, i, nv) in enumerate(serving_requests(args.requests, seed,
                                                        rate)):
            f, g = pools[i]
            out.append(Request(k, f"s{i}", f[:nv], t, out=g[:nv]))
        return out

    levels = {}
    sat = summarize(srv.run(stream(None, 4)), Ns.get)
    rate_sat = sat["served"] / sat["span_s"]
    levels["saturation"] = dict(sat, rate_rps=rate_sat)
    print(json.dumps({"level": "saturation", **levels["saturation"]}),
          file=sys.stderr, flush=True)
    for frac in (0.5, 0.8, 1.2):
        st = summarize(srv.run(stream(frac * rate_sat, 4)), Ns.get)
        levels[f"{frac}x"] = dict(st, rate_rps=frac * rate_sat)
        print(json.dumps({"level": frac, **st}), file=sys.stderr, flush=True)
    sizes = [nv for _, nv in srv.batches]
    out = {
        "metric": "serving: N·nvec/s at saturation",
        "value": sat["throughput"],
        "unit": "N·nvec/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": 0,
        "ms_per_step": sat["span_s"] * 1e3 / max(1, sat["served"]),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving_mix", "plans": len(SERVING_SHAPES),
                   "requests_per_level": args.requests,
                   "max_batch": max_batch},
        "levels": levels,
        "batches": len(sizes),
        "device_overlap": overlap_fraction(srv.intervals),
        "mean_batch_vectors": float(np.mean(sizes)) if sizes else 0.0,
        "resident_plan_bytes": srv.cache.resident_bytes,
        "plan_builds": srv.cache.builds,
        "plan_evictions": srv.cache.evictions,
        "plan_build_s": build_s,
    }
    srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
