"""Host-side checks of libbf.so that need no GPU: the library loads, exports
every symbol include/bf.h declares, its plan geometry matches the oracle's
(independently written) geometry, and argument errors are reported through
status codes."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1803_04128_amd as bfm
from paper_1803_04128_amd import _lib
from oracle.butterfly import mock_chebyshev, lagrange_1d

HEADER = os.path.join(os.path.dirname(os.path.dirname(
    os.path.abspath(__file__))), "include", "bf.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(bf_\w+)\s*\(",
                                 src, re.M)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert "bf_plan" in names and "bf_apply" in names and len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTS)


@pytest.mark.parametrize("q", range(2, 17))
def test_points_match_oracle(q):
    for L in range(0, 23):
        size = 1 << L
        assert np.array_equal(bfm.points(size, q), mock_chebyshev(size, q)), \
            (size, q)


@pytest.mark.parametrize("size,q", [(16, 8), (1024, 10), (64, 7), (8, 5)])
def test_lagrange_matches_oracle(size, q):
    nodes = mock_chebyshev(size, q)
    y = np.arange(-3, 2 * size + 3, dtype=float)
    ours = bfm.lagrange(nodes, y)
    ref = lagrange_1d(nodes, y)
    assert np.allclose(ours, ref, rtol=1e-13, atol=1e-13)


def _plan_rc(dim=1, n=64, kind=1, params=(2.0, 1.0, 8.0), q=8, prec=0,
             max_nvec=1, amp=None):
    lib = _lib.load()
    g = _lib.BfGrid(dim, n)
    arr = (C.c_double * max(1, len(params)))(*params)
    ph = _lib.BfPhase(kind, len(params), arr)
    h = C.c_void_p()
    rc = lib.bf_plan(C.byref(g), C.byref(ph), C.byref(amp) if amp else None,
                     q, prec, max_nvec, C.byref(h))
    return rc, h


@pytest.mark.parametrize("kw", [
    dict(dim=3), dict(n=100), dict(n=1), dict(q=1), dict(q=17),
    dict(dim=2, n=16, kind=2, params=(2, 1, 16, 2, 1, 16), q=9),
    dict(prec=7), dict(max_nvec=0), dict(kind=9), dict(params=(1.0,)),
    dict(kind=2, params=(2, 1, 16, 2, 1, 16)),   # radon phase needs 2D
])
def test_plan_rejects_bad_arguments(kw):
    rc, h = _plan_rc(**kw)
    assert rc == _lib.BF_EINVAL
    assert not h.value
    assert len(_lib.load().bf_last_error()) > 0


def test_amplitude_arguments_checked():
    a = np.ones(2 * 64, np.float64)
    amp = _lib.BfAmplitude(2, None, None)          # alpha = 1 needs r = 1
    rc, _ = _plan_rc(amp=amp)
    assert rc == _lib.BF_EINVAL
    amp = _lib.BfAmplitude(1, a.ctypes.data_as(C.POINTER(C.c_double)), None)
    rc, _ = _plan_rc(amp=amp)
    assert rc == _lib.BF_EINVAL


def test_null_handles():
    lib = _lib.load()
    assert lib.bf_destroy(None) == _lib.BF_OK
    assert lib.bf_apply(None, 1, None, None, None) == _lib.BF_EINVAL
    info = _lib.BfPlanInfo()
    assert lib.bf_query(None, C.byref(info)) == _lib.BF_EINVAL
    sz = C.c_size_t()
    assert lib.bf_workspace_bytes(None, 1, C.byref(sz)) == _lib.BF_EINVAL


def test_no_device_is_an_error_not_a_crash():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h = _plan_rc()
    assert rc in (_lib.BF_EHIP, _lib.BF_ENOMEM)
    assert not h.value


_RADON16 = dict(dim=2, n=16, kind=2, params=(2, 1, 16, 2, 1, 16), q=7)


@pytest.mark.parametrize("prec", [1, 2])
def test_split_precision_2d_planned_up_to_device_use(prec):
    """2D split plans pass every host check: without a GPU they fail only
    where the device is first needed, like an FP32 plan."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h = _plan_rc(prec=prec, **_RADON16)
    assert rc in (_lib.BF_EHIP, _lib.BF_ENOMEM)
    assert not h.value


@pytest.mark.parametrize("env", ["BF_SWITCH_OTF", "BF_MFMA"])
def test_split_precision_2d_forms_refused_before_device_use(env, monkeypatch):
    """The split forms of a 2D plan are the per-step MFMA kernels with
    stored switch blocks: on-the-fly switch evaluation or the scalar
    per-step kernels are refused at plan time."""
    monkeypatch.setenv(env, "1" if env == "BF_SWITCH_OTF" else "0")
    rc, h = _plan_rc(prec=1, **_RADON16)
    assert rc == _lib.BF_EUNSUPPORTED
    assert not h.value
    assert b"split" in _lib.load().bf_last_error().lower()


@pytest.mark.parametrize("op", [-1, 4, 7])
def test_plan_op_rejects_unknown_op(op):
    lib = _lib.load()
    g = _lib.BfGrid(1, 64)
    params = (C.c_double * 3)(2.0, 1.0, 8.0)
    ph = _lib.BfPhase(1, 3, params)
    h = C.c_void_p()
    rc = lib.bf_plan_op(C.byref(g), C.byref(ph), None, 8, 0, 1, op,
                        C.byref(h))
    assert rc == _lib.BF_EINVAL
    assert not h.value
    assert b"op" in lib.bf_last_error()


def test_python_plan_rejects_unknown_op():
    import paper_1803_04128_amd as bfm
    with pytest.raises(ValueError):
        bfm.Plan(1, 64, "fio1d", (2.0, 1.0, 8.0), q=8, op="X")


def test_apply_chain_rejects_empty_chain():
    lib = _lib.load()
    arr = (C.c_void_p * 1)(None)
    assert lib.bf_apply_chain(None, 1, 1, None, None, None,
                              None) == _lib.BF_EINVAL
    assert lib.bf_apply_chain(arr, 0, 1, None, None, None,
                              None) == _lib.BF_EINVAL


@pytest.mark.parametrize("rank,have_u,have_v", [(0, True, True),
                                                (65, True, True),
                                                (4, False, True),
                                                (4, True, False)])
def test_lowrank_phase_arguments_checked(rank, have_u, have_v):
    lib = _lib.load()
    n = 64
    U = np.zeros((n, max(rank, 1)))
    g = _lib.BfGrid(1, n)
    dp = C.POINTER(C.c_double)
    ph = _lib.BfPhase(5, 0, None, rank,
                      U.ctypes.data_as(dp) if have_u else None,
                      U.ctypes.data_as(dp) if have_v else None)
    h = C.c_void_p()
    rc = lib.bf_plan(C.byref(g), C.byref(ph), None, 8, 0, 1, C.byref(h))
    assert rc == _lib.BF_EINVAL
    assert not h.value
