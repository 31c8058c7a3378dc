"""MI355X (gfx950) interpolative butterfly apply for oscillatory transforms.

g = K f with K(x, xi) = alpha(x, xi) exp(2 pi i Phi(x, xi)), computed as
g = sum_k a_k * BF(b_k * f) (eq. (eqn:tg) of arXiv:1803.04128) with the
butterfly factorization of Section 4.  This module is a thin ctypes binding
of libbf.so (include/bf.h): it marshals arguments; every step of the apply
runs in the library's HIP kernels.  PyTorch provides device memory and
streams only.
"""

import ctypes as C

import numpy as np

from . import _lib
from ._lib import BfError, OPS, PATHS, PHASES, PRECISIONS  # noqa: F401

__all__ = ["Plan", "Graph", "BfError", "points", "lagrange", "load",
           "plan_footprint", "lift_decide", "plan_lifted", "plan_for_kernel",
           "apply_chain", "graph_chain", "fourier_coefficients_plan",
           "unwrap",
           "recover_phase", "kernel_phase_sampler", "lowrank_from_samples",
           "kernel_samples", "recover_kernel"]


def load():
    return _lib.load()


def points(box_size, q):
    """Host-only: 0-based interpolation offsets of a box (bf_points)."""
    lib = _lib.load()
    out = (C.c_int * 16)()
    cnt = C.c_int()
    _lib.check(lib.bf_points(int(box_size), int(q), out, 16, C.byref(cnt)))
    return np.array(out[:cnt.value], dtype=np.int64)


def lagrange(nodes, y):
    """Host-only: Lagrange weights [len(y)][len(nodes)] (bf_lagrange)."""
    lib = _lib.load()
    nodes = np.ascontiguousarray(nodes, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros((y.size, nodes.size), np.float64)
    _lib.check(lib.bf_lagrange(
        nodes.ctypes.data_as(C.POINTER(C.c_int)), nodes.size,
        y.ctypes.data_as(C.POINTER(C.c_double)), y.size,
        out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def _plan_structs(dim, n, phase, params, amplitude, op):
    """The bf_grid, bf_phase and bf_amplitude of a plan, and the arrays
    their pointers refer to (keep them alive while the structs are used)."""
    if op not in OPS:
        raise ValueError(f"op must be one of {sorted(OPS)}")
    grid = _lib.BfGrid(int(dim), int(n))
    if phase == "lowrank":
        # params = (U, V): real factors [N][rank], Phi = U V^T
        U, V = (np.ascontiguousarray(m, dtype=np.float64) for m in params)
        if U.ndim != 2 or U.shape != V.shape or U.shape[0] != n ** dim:
            raise ValueError("low-rank phase factors must both be "
                             "[N][rank]")
        pa = (C.c_double * 1)()
        ph = _lib.BfPhase(PHASES[phase], 0, pa, U.shape[1],
                          U.ctypes.data_as(C.POINTER(C.c_double)),
                          V.ctypes.data_as(C.POINTER(C.c_double)))
        keep = [pa, U, V]
    else:
        pa = (C.c_double * max(1, len(params)))(*params)
        ph = _lib.BfPhase(PHASES[phase], len(params), pa)
        keep = [pa]
    amp = None
    if amplitude is not None:
        a, b = amplitude
        a = np.ascontiguousarray(a, dtype=np.complex128)
        b = np.ascontiguousarray(b, dtype=np.complex128)
        if a.shape != b.shape or a.ndim != 2 or a.shape[1] != n ** dim:
            raise ValueError("amplitude factors must both be [r][N]")
        amp = _lib.BfAmplitude(
            a.shape[0], a.ctypes.data_as(C.POINTER(C.c_double)),
            b.ctypes.data_as(C.POINTER(C.c_double)))
        keep += [a, b]
    return grid, ph, amp, keep


def plan_footprint(dim, n, phase, params=(), q=8, amplitude=None,
                   precision="fp32", max_nvec=1, op="N"):
    """Device bytes Plan(...) with these arguments would allocate (factors,
    stored switch blocks, low-rank phase factors, workspace), computed on
    the host without touching a device (bf_plan_footprint)."""
    lib = _lib.load()
    grid, ph, amp, keep = _plan_structs(dim, n, phase, params, amplitude, op)
    out = C.c_size_t()
    _lib.check(lib.bf_plan_footprint(
        C.byref(grid), C.byref(ph), C.byref(amp) if amp else None, int(q),
        PRECISIONS[precision], int(max_nvec), OPS[op], C.byref(out)))
    del keep
    return out.value


def lift_decide(U1, V1, U2, V2, r, r_eps, eps, omega, test_cols,
                alg1_samples):
    """Algorithm 6 (bf_lift_decide), host only: whether the kernel with
    phase U1 V1^T and amplitude U2 V2^T (real [N][r1], [N][r2]) can be
    applied as r_eps r-dimensional NUFFTs after lifting its phase to rank r.
    omega [N][m] (m > r1), test_cols and alg1_samples = (row rounds [t][s],
    column rounds [t][s], extra rows, extra columns) are the method's random
    draws.  Returns (y, n, P, Q, a, b): a, b complex [k][N] when y = 1, else
    None."""
    lib = _lib.load()
    f64 = lambda m: np.ascontiguousarray(m, dtype=np.float64)  # noqa: E731
    i64 = lambda m: np.ascontiguousarray(m, dtype=np.int64)    # noqa: E731
    U1, V1, U2, V2, omega = (f64(m) for m in (U1, V1, U2, V2, omega))
    N, r1 = U1.shape
    r2 = U2.shape[1]
    if V1.shape != U1.shape or V2.shape != U2.shape or U2.shape[0] != N or \
            omega.ndim != 2 or omega.shape[0] != N:
        raise ValueError("factors must be [N][rank] and omega [N][m]")
    tc = i64(test_cols)
    rows, cols, xr, xc = alg1_samples
    rows, cols = i64(rows), i64(cols)
    xr, xc = i64(xr), i64(xc)
    if rows.ndim != 2 or rows.shape != cols.shape or xr.shape != xc.shape:
        raise ValueError("alg1_samples: rounds [t][s] of rows and columns, "
                         "extra rows and columns of one length")
    P = np.zeros((N, r))
    Q = np.zeros((N, r))
    a = np.zeros((r_eps, N), np.complex128)
    b = np.zeros((r_eps, N), np.complex128)
    y, n, k = C.c_int(), C.c_int(), C.c_int()
    D, L = C.POINTER(C.c_double), C.POINTER(C.c_longlong)
    _lib.check(lib.bf_lift_decide(
        N, r1, U1.ctypes.data_as(D), V1.ctypes.data_as(D), r2,
        U2.ctypes.data_as(D), V2.ctypes.data_as(D), int(r), int(r_eps),
        float(eps), omega.ctypes.data_as(D), omega.shape[1],
        tc.ctypes.data_as(L), tc.size, rows.shape[0], rows.ctypes.data_as(L),
        cols.ctypes.data_as(L), rows.shape[1], xr.ctypes.data_as(L),
        xc.ctypes.data_as(L), xr.size, C.byref(y), C.byref(n),
        P.ctypes.data_as(D), Q.ctypes.data_as(D), a.ctypes.data_as(D),
        b.ctypes.data_as(D), C.byref(k)))
    if not y.value:
        return 0, n.value, P, Q, None, None
    return 1, n.value, P, Q, a[:k.value].copy(), b[:k.value].copy()


def plan_lifted(P, Q, a, b, max_nvec=1):
    """A device plan of eq. (eqn:tg3) (bf_plan_lifted): g = sum_k a_k .
    NUFFT3(P, Q; b_k . f).  P, Q real [N][r], a, b complex [k][N]."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    if P.ndim != 2 or P.shape != Q.shape or a.shape != b.shape or \
            a.ndim != 2 or a.shape[1] != P.shape[0]:
        raise ValueError("P, Q must be [N][r] and a, b [k][N]")
    return Plan._from_lifted(P, Q, a, b, max_nvec)


def plan_for_kernel(U1, V1, U2, V2, r, r_eps, eps, omega, test_cols,
                    alg1_samples, q=8, max_nvec=1):
    """The unified framework (Figure (fig:flow), 1D): Algorithm 6 decides,
    then the NUFFT path (plan_lifted) or the butterfly of the low-rank
    phase with the amplitude factors (Plan with phase "lowrank").  Returns
    (plan, decision) with decision = (y, n)."""
    y, n, P, Q, a, b = lift_decide(U1, V1, U2, V2, r, r_eps, eps, omega,
                                   test_cols, alg1_samples)
    if y:
        return plan_lifted(P, Q, a, b, max_nvec), (y, n)
    U1 = np.asarray(U1, np.float64)
    N = U1.shape[0]
    amp = (np.asarray(U2, np.float64).T.astype(np.complex128),
           np.asarray(V2, np.float64).T.astype(np.complex128))
    if amp[0].shape[0] == 1 and np.all(amp[0] == 1) and np.all(amp[1] == 1):
        amp = None
    return Plan(1, N, "lowrank", (U1, V1), q=q, amplitude=amp,
                max_nvec=max_nvec), (y, n)


class Plan:
    """A device-resident butterfly plan (bf_plan ... bf_destroy).

    dim, n: grid (x_i = i/n, xi_j = j - n/2 per dimension).
    phase: "dft" | "fio1d" | "fio1d_warp" | "radon2d" | "separable" with
    params its numbers, or "lowrank" with params = (U, V), real [N][rank]
    factors of Phi = U V^T.
    q: interpolation points per box and dimension.
    amplitude: None (alpha = 1) or (a, b), complex arrays [r][N].
    precision: "fp32" | "bf16x3" | "fp16x3".
    op: "N" (K), "T" (K^T), "C" (entrywise conjugate) or "H" (K^H): the
    operator apply() computes (Scenario 2 of Section 1); a, b keep their
    meaning (a_k on the x grid, b_k on the xi grid).
    """

    def __init__(self, dim, n, phase, params=(), q=8, amplitude=None,
                 precision="fp32", max_nvec=1, op="N"):
        self._lib = _lib.load()
        self._h = C.c_void_p()
        grid, ph, amp, self._keep = _plan_structs(dim, n, phase, params,
                                                  amplitude, op)
        self.r = amp.r if amp is not None else 1
        _lib.check(self._lib.bf_plan_op(
            C.byref(grid), C.byref(ph), C.byref(amp) if amp else None,
            int(q), PRECISIONS[precision], int(max_nvec), OPS[op],
            C.byref(self._h)))
        import torch
        # bf_plan builds on the current device; applies must stay there
        self.device = torch.cuda.current_device()
        self.op = op
        self.dim, self.n, self.q = dim, n, q
        self.N = n ** dim
        self.max_nvec = max_nvec
        self.precision = precision

    @classmethod
    def _from_lifted(cls, P, Q, a, b, max_nvec):
        import torch
        self = cls.__new__(cls)
        self._lib = _lib.load()
        self._h = C.c_void_p()
        D = C.POINTER(C.c_double)
        N, r = P.shape
        _lib.check(self._lib.bf_plan_lifted(
            N, r, P.ctypes.data_as(D), Q.ctypes.data_as(D), a.shape[0],
            a.ctypes.data_as(D), b.ctypes.data_as(D), int(max_nvec),
            C.byref(self._h)))
        self._keep = []
        self.device = torch.cuda.current_device()
        self.r = a.shape[0]
        self.op = "N"
        self.dim, self.n, self.q = 1, N, 0
        self.N = N
        self.max_nvec = max_nvec
        self.precision = "fp32"
        return self

    def info(self):
        inf = _lib.BfPlanInfo()
        _lib.check(self._lib.bf_query(self._h, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def steps(self):
        """The computed steps (bf_step_query): kind, level, ranks, stored
        entry counts."""
        out = []
        for k in range(self.info()["n_steps"]):
            si = _lib.BfStepInfo()
            _lib.check(self._lib.bf_step_query(self._h, k, C.byref(si)))
            out.append({n: getattr(si, n) for n, _ in si._fields_})
        return out

    def factor_entries(self, step, which, idx):
        """Stored factor entries of a step (bf_factor_entries): which is
        "twiddle" or "switch"; returns (x [count][3], xi [count][3] user
        indices of the phase terms, -1 past the last; complex64 values)."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        n = idx.size
        x = np.empty((n, 3), np.int64)
        xi = np.empty((n, 3), np.int64)
        v = np.empty(2 * n, np.float32)
        lp = C.POINTER(C.c_longlong)
        _lib.check(self._lib.bf_factor_entries(
            self._h, int(step), {"twiddle": 0, "switch": 1}[which],
            idx.ctypes.data_as(lp), n, x.ctypes.data_as(lp),
            xi.ctypes.data_as(lp), v.ctypes.data_as(C.POINTER(C.c_float))))
        return x, xi, v.view(np.complex64).copy()

    def workspace_bytes(self, nvec):
        v = C.c_size_t()
        _lib.check(self._lib.bf_workspace_bytes(self._h, int(nvec),
                                                C.byref(v)))
        return v.value

    @staticmethod
    def _stream(stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        return C.c_void_p(s.cuda_stream)

    def _device_tensor(self, t, name, complex64=True):
        """Reject what the kernels must not see: host tensors (whose host
        pointer would reach the GPU), tensors on another device, other
        dtypes and non-contiguous views."""
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.device.index != self.device:
            raise ValueError(f"{name} is on cuda:{t.device.index}, the plan "
                             f"on cuda:{self.device}")
        if complex64 and t.dtype != torch.complex64:
            raise TypeError(f"{name} must be complex64")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _args(self, f, out):
        import torch
        self._device_tensor(f, "f")
        f2 = f.reshape(1, -1) if f.dim() == 1 else f
        if f2.dim() != 2 or f2.shape[-1] != self.N:
            raise ValueError("f must be [nvec][N] (or [N])")
        if out is None:
            out = torch.empty_like(f2)
        else:
            self._device_tensor(out, "out")
            if out.dim() == 1:
                out = out.reshape(1, -1)
        if out.shape != f2.shape:
            raise ValueError("out must have the shape of f")
        return f2, out, f2.shape[0]

    def apply(self, f, out=None, stream=None, workspace=None):
        """g = K f for a complex64 CUDA tensor f [nvec][N] (or [N]).
        Asynchronous on ``stream`` (default: torch's current stream)."""
        squeeze = f.dim() == 1
        f2, out, nvec = self._args(f, out)
        if workspace is not None:
            self._device_tensor(workspace, "workspace", complex64=False)
        st = self._stream(stream)
        if workspace is None:
            _lib.check(self._lib.bf_apply(self._h, nvec, C.c_void_p(
                f2.data_ptr()), C.c_void_p(out.data_ptr()), st))
        else:
            _lib.check(self._lib.bf_apply_ws(
                self._h, nvec, C.c_void_p(f2.data_ptr()),
                C.c_void_p(out.data_ptr()), C.c_void_p(workspace.data_ptr()),
                workspace.numel() * workspace.element_size(), st))
        return out.reshape(-1) if squeeze else out

    def apply_static(self, f, out=None, stream=None):
        """As apply(), through the allocation-free entry point
        (bf_apply_static): the workspace is the library's static device
        buffer of each GPU, shared by every such call on that GPU, so calls
        that overlap in time on one GPU race.  out is allocated by torch
        when not given (pass it for an allocation-free call)."""
        squeeze = f.dim() == 1
        f2, out, nvec = self._args(f, out)
        _lib.check(self._lib.bf_apply_static(
            self._h, nvec, C.c_void_p(f2.data_ptr()),
            C.c_void_p(out.data_ptr()), self._stream(stream)))
        return out.reshape(-1) if squeeze else out

    def config(self):
        """Execution form: {"path", "tile_cols", "tile_cols_used",
        "switch_otf", "max_pass_levels", "twiddle_otf"}."""
        c = _lib.BfConfig()
        _lib.check(self._lib.bf_get_config(self._h, C.byref(c)))
        names = {v: k for k, v in PATHS.items()}
        return dict(path=names[c.path], tile_cols=c.tile_cols,
                    tile_cols_used=c.tile_cols_used,
                    switch_otf=bool(c.switch_otf),
                    max_pass_levels=c.max_pass_levels,
                    twiddle_otf=bool(c.twiddle_otf))

    def set_config(self, path="fused", tile_cols=0, switch_otf=False,
                   max_pass_levels=0, twiddle_otf=False):
        """switch_otf (per_step_mfma only): generate the switch blocks
        during the apply instead of storing them.  max_pass_levels (fused
        forms): at most this many levels per pass, each half split into
        equal passes (0: as many as the LDS holds).  twiddle_otf
        (per_step_mfma, FP32): evaluate the twiddles during the apply, as
        stored, instead of reading them."""
        c = _lib.BfConfig(PATHS[path], int(tile_cols), 0,
                          1 if switch_otf else 0, int(max_pass_levels),
                          1 if twiddle_otf else 0)
        _lib.check(self._lib.bf_set_config(self._h, C.byref(c)))

    def autotune(self, f, out=None, reps=3, stream=None):
        """Time the candidate execution forms on f (bf_autotune) and keep
        the fastest; returns the candidates with their ms per apply."""
        f2, out, nvec = self._args(f, out)
        cap = 32
        arr = (_lib.BfTuneEntry * cap)()
        cnt = C.c_int()
        _lib.check(self._lib.bf_autotune(
            self._h, nvec, C.c_void_p(f2.data_ptr()),
            C.c_void_p(out.data_ptr()), int(reps), self._stream(stream), arr,
            cap, C.byref(cnt)))
        names = {v: k for k, v in PATHS.items()}
        return [dict(path=names[e.config.path], tile_cols=e.config.tile_cols,
                     tile_cols_used=e.config.tile_cols_used,
                     switch_otf=bool(e.config.switch_otf),
                     max_pass_levels=e.config.max_pass_levels,
                     twiddle_otf=bool(e.config.twiddle_otf), ms=e.ms)
                for e in arr[:min(cnt.value, cap)]]

    def graph(self, f, out=None):
        """Capture the apply on f into a replayable HIP graph."""
        return Graph(self, f, out)

    def profile(self, enable=True):
        """Start (or stop) per-launch event timing inside the library."""
        _lib.check(self._lib.bf_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """Per-kernel-class totals since the last read (synchronises)."""
        cap = 64
        arr = (_lib.BfKernelStat * cap)()
        cnt = C.c_int()
        _lib.check(self._lib.bf_profile_read(self._h, arr, cap,
                                             C.byref(cnt)))
        out = {}
        for k in arr[:min(cnt.value, cap)]:
            out[k.name.decode()] = dict(launches=k.launches,
                                        total_ms=k.total_ms, bytes=k.bytes,
                                        flops=k.flops,
                                        state_bytes=k.state_bytes)
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(self._lib.bf_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Graph:
    """A captured apply (bf_graph_create) or chain (bf_graph_create_chain):
    replays it for the tensors it was built with, in one launch call.  Keep
    f, out (and tmp) alive while it exists."""

    def __init__(self, plan, f, out=None, chain=None, tmp=None):
        self._lib = plan._lib
        self.plan = plan
        self.f, self.out, nvec = plan._args(f, out)
        self._h = C.c_void_p()
        if chain is None:
            _lib.check(self._lib.bf_graph_create(
                plan._h, nvec, C.c_void_p(self.f.data_ptr()),
                C.c_void_p(self.out.data_ptr()), C.byref(self._h)))
            return
        import torch
        if tmp is not None:
            plan._device_tensor(tmp, "tmp")
            if tmp.numel() != self.f.numel():
                raise ValueError("tmp must have the shape of f")
        self.tmp = tmp if tmp is not None or len(chain) == 1 else \
            torch.empty_like(self.f)
        arr = (C.c_void_p * len(chain))(*[p._h.value for p in chain])
        _lib.check(self._lib.bf_graph_create_chain(
            arr, len(chain), nvec, C.c_void_p(self.f.data_ptr()),
            C.c_void_p(self.out.data_ptr()),
            C.c_void_p(self.tmp.data_ptr() if self.tmp is not None
                       else None), C.byref(self._h)))

    def launch(self, stream=None):
        _lib.check(self._lib.bf_graph_launch(self._h,
                                             Plan._stream(stream)))
        return self.out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(self._lib.bf_graph_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def apply_chain(plans, f, out=None, tmp=None, stream=None):
    """g = P_m(... P_2(P_1 f)) through bf_apply_chain, e.g. the composition
    of two FIOs of eq. (eq:example4) as [L, F, L] with F from
    fourier_coefficients_plan.  tmp: an optional complex64 tensor like f
    for the intermediate results (allocated when not given)."""
    plans = list(plans)
    if not plans:
        raise ValueError("apply_chain needs at least one plan")
    squeeze = f.dim() == 1
    f2, out, nvec = plans[0]._args(f, out)
    if tmp is None and len(plans) > 1:
        import torch
        tmp = torch.empty_like(f2)
    if tmp is not None:
        plans[0]._device_tensor(tmp, "tmp")
        if tmp.numel() != f2.numel():
            raise ValueError("tmp must have the shape of f")
    arr = (C.c_void_p * len(plans))(*[p._h.value for p in plans])
    _lib.check(plans[0]._lib.bf_apply_chain(
        arr, len(plans), nvec, C.c_void_p(f2.data_ptr()),
        C.c_void_p(out.data_ptr()),
        C.c_void_p(tmp.data_ptr() if tmp is not None else None),
        Plan._stream(stream)))
    return out.reshape(-1) if squeeze else out


def graph_chain(plans, f, out=None, tmp=None):
    """Capture apply_chain(plans, f) into one HIP graph
    (bf_graph_create_chain); launch() replays it."""
    plans = list(plans)
    return Graph(plans[0], f, out, chain=plans, tmp=tmp)


def fourier_coefficients_plan(n, q=10, precision="fp32", max_nvec=1):
    """The plan of hat_j = (1/n) sum_i h_i exp(-2 pi i x_i xi_j): the
    adjoint of the DFT-phase kernel with the constant amplitude 1/n, which
    turns the grid values one FIO of eq. (eq:example3) produces into the
    coefficients the next one takes."""
    a = np.full((1, n), 1.0 / n, np.complex128)
    b = np.ones((1, n), np.complex128)
    return Plan(1, n, "dft", (), q=q, amplitude=(a, b), precision=precision,
                max_nvec=max_nvec, op="H")


def unwrap(u, tau=np.pi / 2):
    """Algorithm 3 (bf_unwrap): v equal to u modulo 1 with matched second
    differences, and the restart (discontinuity) indices."""
    lib = _lib.load()
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.empty_like(u)
    cap = 64
    disc = (C.c_longlong * cap)()
    nd = C.c_int()
    dp = C.POINTER(C.c_double)
    _lib.check(lib.bf_unwrap(u.ctypes.data_as(dp), u.size, float(tau),
                             v.ctypes.data_as(dp), disc, cap, C.byref(nd)))
    if nd.value > cap:
        raise RuntimeError("more restarts than the buffer holds")
    return v, np.asarray(disc[:nd.value], np.int64)


def recover_phase(N, C_idx, R_idx, sampler, rank=8, tau=np.pi / 2):
    """Algorithm 5 (bf_recover_phase) for a 1D phase known modulo 1 through
    sampler(is_row, idx) -> [N][len(idx)] (columns) or [len(idx)][N] (rows),
    phases in cycles.  C_idx, R_idx: the sampled column and row indices
    (the caller's random choice).  Returns U, V [N][k] with exp(2 pi i U
    V^T) = exp(2 pi i Phi), for Plan(..., "lowrank", (U, V))."""
    lib = _lib.load()
    Ci = np.ascontiguousarray(np.unique(C_idx), dtype=np.int64)
    Ri = np.ascontiguousarray(np.unique(R_idx), dtype=np.int64)
    failure = []

    def cb(ctx, is_row, count, idx, out):
        try:
            ids = np.ctypeslib.as_array(idx, shape=(count,)).copy()
            vals = np.asarray(sampler(bool(is_row), ids), np.float64)
            want = (count, N) if is_row else (N, count)
            if vals.shape != want:
                raise ValueError(f"sampler returned {vals.shape}, "
                                 f"expected {want}")
            np.ctypeslib.as_array(out, shape=(count * N,))[:] = vals.ravel()
            return 0
        except Exception as e:          # reported after the call
            failure.append(e)
            return 1

    cfun = _lib.SAMPLER(cb)
    cap = int(rank)
    U = np.zeros((N, cap))
    V = np.zeros((N, cap))
    k = C.c_int()
    lp = C.POINTER(C.c_longlong)
    dp = C.POINTER(C.c_double)
    rc = lib.bf_recover_phase(int(N), Ci.ctypes.data_as(lp), Ci.size,
                              Ri.ctypes.data_as(lp), Ri.size, int(rank),
                              float(tau), cfun, None, cap,
                              U.ctypes.data_as(dp), V.ctypes.data_as(dp),
                              C.byref(k))
    if failure:
        raise failure[0]
    _lib.check(rc)
    return U[:, :k.value].copy(), V[:, :k.value].copy()


def lowrank_from_samples(N, cols, C_idx, rows, R_idx, rank=8):
    """Algorithm 1 on given samples of a real N x N matrix A
    (bf_lowrank_samples): cols [N][len(C_idx)] = A(:, C_idx), rows
    [len(R_idx)][N] = A(R_idx, :), indices sorted and distinct.  Returns
    U, V [N][k] with A ~ U V^T."""
    lib = _lib.load()
    Ci = np.ascontiguousarray(C_idx, dtype=np.int64)
    Ri = np.ascontiguousarray(R_idx, dtype=np.int64)
    cols_t = np.ascontiguousarray(np.asarray(cols, np.float64).T)
    rows_c = np.ascontiguousarray(rows, dtype=np.float64)
    if cols_t.shape != (Ci.size, N) or rows_c.shape != (Ri.size, N):
        raise ValueError("cols must be [N][len(C)] and rows [len(R)][N]")
    cap = int(rank)
    U = np.zeros((N, cap))
    V = np.zeros((N, cap))
    k = C.c_int()
    lp = C.POINTER(C.c_longlong)
    dp = C.POINTER(C.c_double)
    _lib.check(lib.bf_lowrank_samples(
        int(N), cols_t.ctypes.data_as(dp), Ci.ctypes.data_as(lp), Ci.size,
        rows_c.ctypes.data_as(dp), Ri.ctypes.data_as(lp), Ri.size, int(rank),
        cap, U.ctypes.data_as(dp), V.ctypes.data_as(dp), C.byref(k)))
    return U[:, :k.value].copy(), V[:, :k.value].copy()


def kernel_samples(plan, plan_t, idx, rows):
    """Columns K e_j (rows=False; [N][len(idx)]) or rows K^T e_i (rows=True;
    [len(idx)][N]) of the kernel from applies of ``plan`` and of
    ``plan_t`` (a BF_OP_T plan of the same kernel) to unit vectors."""
    import torch
    N = plan.N
    pl = plan_t if rows else plan
    out = np.empty((len(idx), N), np.complex128)
    step = pl.max_nvec
    for s in range(0, len(idx), step):
        part = np.asarray(idx[s:s + step])
        e = torch.zeros((len(part), N), dtype=torch.complex64, device="cuda")
        e[torch.arange(len(part)), torch.as_tensor(part)] = 1.0
        out[s:s + len(part)] = pl.apply(e).cpu().numpy()
    return out if rows else out.T


def recover_kernel(plan, plan_t, C_idx, R_idx, amp_rank=4, phase_rank=4,
                   tau=np.pi / 2):
    """Scenario 2 of Table (tab:sc), 1D: from applies of K and K^T only,
    the amplitude's low-rank factors (Algorithm 1 on |K|) and the phase's
    (Algorithm 5 on arg K, the amplitude being positive).  Returns
    ((a, b), (U, V)): a, b complex [k][N] for Plan(amplitude=(a, b)) and
    U, V for Plan(phase="lowrank", params=(U, V))."""
    N = plan.N
    Ci = np.unique(np.asarray(C_idx, np.int64))
    Ri = np.unique(np.asarray(R_idx, np.int64))
    cols = np.abs(kernel_samples(plan, plan_t, Ci, rows=False))
    rows = np.abs(kernel_samples(plan, plan_t, Ri, rows=True))
    # rows and columns must agree where they meet: take the row samples
    # there (both are the same entries of |K| up to the applies' rounding)
    cols[Ri, :] = rows[:, Ci]
    Ua, Va = lowrank_from_samples(N, cols, Ci, rows, Ri, amp_rank)
    U, V = recover_phase(N, Ci, Ri, kernel_phase_sampler(plan, plan_t),
                         rank=phase_rank, tau=tau)
    return ((Ua.T.astype(np.complex128), Va.T.astype(np.complex128)),
            (U, V))


def kernel_phase_sampler(plan, plan_t, amplitude=None):
    """Scenario 2 sampler for recover_phase: the columns of K are K e_j
    (applies of ``plan``), its rows K^T e_i (applies of ``plan_t``, a
    BF_OP_T plan of the same kernel); the phase in cycles is arg(K / alpha)
    / (2 pi), which for a positive amplitude is arg(K) / (2 pi).
    amplitude: None or a callable (is_row, idx) -> alpha on the same
    samples."""
    def sample(is_row, idx):
        k = kernel_samples(plan, plan_t, idx, rows=is_row)
        if amplitude is not None:
            k = k / np.asarray(amplitude(is_row, idx))
        return np.angle(k) / (2 * np.pi)
    return sample

