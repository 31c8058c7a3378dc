"""The allocation-free apply (bf_apply_static), through the C ABI: its
results match bf_apply's on the same plan to the FP32 bar (1e-5 relative
l2 per vector; the static buffer may hold fewer vectors per chunk than the
plan's own workspace, which can change the tile width and so the rounding)
and the oracle's butterfly, on two calls in a row, the second with a
smaller input, and neither call changes the device's free memory.  Plans
whose one-vector workspace exceeds the buffer are refused."""

import ctypes as C

import numpy as np
import pytest

from _util import inputs, log, rel
from oracle.butterfly import butterfly_apply, butterfly_matvec
from synthetic import PHASE_PARAMS

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _static(plan, f):
    """bf_apply_static through the C ABI on torch's current stream, with
    the output preallocated; returns (result, free bytes before, after)."""
    import torch
    from paper_1803_04128_amd import _lib
    g = torch.empty_like(f)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    _lib.check(plan._lib.bf_apply_static(
        plan._h, f.shape[0], C.c_void_p(f.data_ptr()),
        C.c_void_p(g.data_ptr()),
        C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return g, free0, free1


@pytest.mark.parametrize("case", [
    # (dim, n, phase, q, amp, r, nvec of the first call, of the second)
    (1, 1 << 14, "fio1d", 8, "sincos", 4, 16, 3),
    (1, 1 << 18, "fio1d", 10, "sincos", 4, 8, 1),
    (2, 128, "radon2d", 7, "one", 1, 6, 2),
])
def test_static_apply_matches_apply_twice(case):
    import torch
    import paper_1803_04128_amd as bfm
    dim, n, phase, q, amp, r, nv1, nv2 = case
    log(f"case static apply {case}")
    f32, f64, ab = inputs(dim, n, nv1, 17, amp, r)
    with bfm.Plan(dim, n, phase, PHASE_PARAMS[phase], q=q, amplitude=ab,
                  max_nvec=nv1) as pl:
        f = torch.from_numpy(f32).to("cuda")
        ref = pl.apply(f).cpu().numpy().astype(np.complex128)
        for nv in (nv1, nv2):
            g, free0, free1 = _static(pl, f[:nv].contiguous())
            g = g.cpu().numpy().astype(np.complex128)
            e = np.max(rel(g, ref[:nv]))
            log(f"  {nv} vectors: static vs bf_apply {e:.3e}, free memory "
                f"{free0} -> {free1}")
            assert e < TOL
            assert free1 == free0
        # the second (smaller) call against the oracle's butterfly
        fo = f64[:nv2]
        if ab is None:
            bf = butterfly_apply(dim, n, phase, PHASE_PARAMS[phase], q, fo)
        else:
            bf = butterfly_matvec(dim, n, phase, PHASE_PARAMS[phase], q,
                                  ab[0], ab[1], fo)
        e = np.max(rel(g, bf))
        log(f"  second call vs oracle butterfly {e:.3e}")
        assert e < TOL


def test_static_apply_refuses_a_plan_larger_than_the_buffer():
    import torch
    import paper_1803_04128_amd as bfm
    from paper_1803_04128_amd import BfError, _lib
    log("case static apply refused: 1D N=2^20 r=4")
    f32, _, ab = inputs(1, 1 << 20, 1, 3, "sincos", 4)
    with bfm.Plan(1, 1 << 20, "fio1d", PHASE_PARAMS["fio1d"], q=10,
                  amplitude=ab, max_nvec=1) as pl:
        assert pl.workspace_bytes(1) > _lib.STATIC_SCRATCH_BYTES
        f = torch.from_numpy(f32).to("cuda")
        with pytest.raises(BfError, match="static scratch"):
            pl.apply_static(f)
