"""GPU tests of the 2D per-step MFMA form with the switch (Algorithm 4.1,
step 4) fused behind the last xi level (eq. (eqn:2) regrouped): the level's
output pairs stay in LDS and are multiplied by their stored blocks S in the
same launch.

The fused launch forms the same FP32 products in the same order as the
separate xi and switch launches (the level's output is exact FP32 in LDS as
it was in HBM), so its results must equal theirs bit for bit; against the
oracle's butterfly of the same operator the FP32 bar 1e-5 applies.  Cases:
the head level as the last xi level (n = 64, 128: it reads f, 16 input and
49 output points, the level's output placed past the stage buffers), a
level between computed levels (n = 256: the output over the input panel),
other phase kinds, the transposed operator, an amplitude of rank 2, column
counts that leave a partial 16-column tile."""

import numpy as np
import pytest

from _util import inputs, rel, log
from oracle.butterfly import butterfly_apply, butterfly_matvec
from synthetic import PHASE_PARAMS

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("n,kind,q,op,r,nvec", [
    (64, "radon2d", 7, "N", 1, 3),
    (128, "radon2d", 7, "T", 2, 5),
    (256, "radon2d", 7, "N", 1, 17),
    (64, "separable", 7, "H", 1, 2),
    (128, "dft", 6, "N", 1, 1),
    (64, "radon2d", 5, "N", 2, 9),
])
def test_fused_switch_matches_separate_launches_and_oracle(
        n, kind, q, op, r, nvec, monkeypatch):
    import paper_1803_04128_amd as bfm
    log(f"case sep-switch n={n} kind={kind} q={q} op={op} r={r} nvec={nvec}")
    f32, f, ab = inputs(2, n, nvec, 4100 + n + q,
                        amp="sincos" if r > 1 else "one", r=r)
    params = PHASE_PARAMS[kind]
    ft = _to_dev(f32)
    outs = {}
    for fuse in ("1", "0"):
        monkeypatch.setenv("BF_SEP_SWITCH", fuse)
        with bfm.Plan(2, n, kind, params, q=q, amplitude=ab, max_nvec=nvec,
                      op=op) as pl:
            assert pl.config()["path"] == "per_step_mfma"
            pl.profile(True)
            outs[fuse] = _host(pl.apply(ft))
            names = set(pl.profile_read())
            pl.profile(False)
        log(f"  BF_SEP_SWITCH={fuse}: kernels {sorted(names)}")
        if fuse == "1":
            assert "xi_sep_switch" in names and "switch_step_mfma" not in names
        else:
            assert "xi_sep_switch" not in names and "switch_step_mfma" in names
    assert np.array_equal(outs["1"], outs["0"])
    t, c = op in ("T", "H"), op in ("C", "H")
    if ab is None:
        ref = butterfly_apply(2, n, kind, params, q, f, transpose=t,
                              conjugate=c)
    else:
        ref = butterfly_matvec(2, n, kind, params, q, ab[0], ab[1], f,
                               transpose=t, conjugate=c)
    e = np.max(rel(outs["1"], ref))
    log(f"  vs oracle {e:.3e}")
    assert e < TOL
