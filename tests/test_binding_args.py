"""The Python binding rejects buffers the kernels must not see before any
library call: host tensors (their host pointers would reach the GPU),
tensors on another device, wrong dtypes, non-contiguous views, and
amplitude factors whose length is not N.  CPU only: the plan object is
made without bf_plan and its library handle fails on any use."""

import numpy as np
import pytest
import torch

import paper_1803_04128_amd as bfm


class _NoLib:
    def __getattr__(self, name):
        raise AssertionError(f"library call {name} reached")


def _fake_plan(N=64, device=0):
    p = object.__new__(bfm.Plan)
    p._lib = _NoLib()
    p._h = None
    p.N = N
    p.device = device
    p.max_nvec = 4
    return p


class _FakeCuda:
    """Stands in for a device tensor in the checks that follow the
    is_cuda test (no GPU here)."""

    def __init__(self, t, index=0):
        self._t = t
        self.is_cuda = True
        self.device = torch.device("cuda", index)
        self.dtype = t.dtype
        self.shape = t.shape

    def is_contiguous(self):
        return self._t.is_contiguous()

    def dim(self):
        return self._t.dim()

    def reshape(self, *s):
        return _FakeCuda(self._t.reshape(*s), self.device.index)

    def numel(self):
        return self._t.numel()


def test_host_tensors_rejected():
    p = _fake_plan()
    f = torch.zeros(2, 64, dtype=torch.complex64)
    with pytest.raises(TypeError, match="f must be a CUDA tensor"):
        p.apply(f)


def test_device_tensor_checks(monkeypatch):
    p = _fake_plan()
    # let the stand-ins pass the isinstance test of _device_tensor
    monkeypatch.setattr(torch, "Tensor", (torch.Tensor, _FakeCuda))
    ok = _FakeCuda(torch.zeros(2, 64, dtype=torch.complex64))
    assert p._device_tensor(ok, "f") is ok
    with pytest.raises(ValueError, match="cuda:1"):
        p._device_tensor(_FakeCuda(torch.zeros(2, 64, dtype=torch.complex64),
                                   1), "out")
    with pytest.raises(TypeError, match="complex64"):
        p._device_tensor(_FakeCuda(torch.zeros(2, 64, dtype=torch.complex128)),
                         "out")
    nc = torch.zeros(64, 2, dtype=torch.complex64).t()
    with pytest.raises(ValueError, match="contiguous"):
        p._device_tensor(_FakeCuda(nc), "tmp")
    # a workspace may have any dtype but must be a contiguous device tensor
    ws = _FakeCuda(torch.zeros(128, dtype=torch.uint8))
    assert p._device_tensor(ws, "workspace", complex64=False) is ws


def test_out_workspace_tmp_on_host_rejected(monkeypatch):
    p = _fake_plan()
    monkeypatch.setattr(torch, "Tensor", (torch.Tensor, _FakeCuda))
    f = _FakeCuda(torch.zeros(2, 64, dtype=torch.complex64))
    host_out = torch.zeros(2, 64, dtype=torch.complex64)
    with pytest.raises(TypeError, match="out must be a CUDA tensor"):
        p._args(f, host_out)
    out = _FakeCuda(torch.zeros(2, 64, dtype=torch.complex64))
    with pytest.raises(TypeError, match="workspace must be a CUDA tensor"):
        p.apply(f, out, stream=object(),
                workspace=torch.zeros(1024, dtype=torch.uint8))
    with pytest.raises(TypeError, match="tmp must be a CUDA tensor"):
        bfm.apply_chain([p, p], f, out, tmp=host_out, stream=object())
    with pytest.raises(ValueError, match="shape of f"):
        p._args(f, _FakeCuda(torch.zeros(1, 64, dtype=torch.complex64)))


def test_amplitude_length_checked_before_the_library():
    a = np.ones((2, 32), np.complex128)
    with pytest.raises(ValueError, match=r"\[r\]\[N\]"):
        bfm.Plan(1, 64, "dft", (), q=8, amplitude=(a, a))
