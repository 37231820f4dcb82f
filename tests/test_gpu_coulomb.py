"""The Coulomb pair on the FP32 matrix cores (batches of 16 or more RHS) against the FP64 oracle and
against the vector-unit GEMVs, and a batch against one of its RHS alone (bitwise)."""
import numpy as np
import pytest
from conftest import say

from oracle import rttda64 as O
from paper_2601_16949_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("o,v,nq,nrhs,precision", [(24, 96, 60, 16, "fp32"), (40, 104, 33, 20, "mixed"),
                                                   (13, 171, 37, 17, "fp32"), (60, 400, 50, 64, "fp32")])
def test_coulomb_mfma_sigma_matches_oracle(gpu_lib, o, v, nq, nrhs, precision):
    import torch

    storage = "f32" if precision == "fp32" else "bf16"
    prob = I.make_problem(I.Shape(o, v, nq, 0.05, storage=storage), 700 + o)
    op = O.Operator.from_problem(prob)
    ctx = gpu_lib.Context(gpu_lib.DeviceProblem(prob, precision), max_rhs=nrhs)
    tun = ctx.get_tuning()
    assert tun["coulomb_path"] == 2 and tun["small_path"] == 2
    c0, c = I.random_state(o, v, nrhs, seed=5)
    dirs = [I.AXES[r % 3] for r in range(nrhs)]
    field = [0.01 * ((r % 5) - 2) for r in range(nrhs)]
    c0d, cd = gpu_lib.to_planes(c0, c)
    _, s_mfma = ctx.sigma(field, dirs, c0d, cd)
    ctx.set_tuning(coulomb_path=1)
    _, s_valu = ctx.sigma(field, dirs, c0d, cd)
    ctx.set_tuning(coulomb_path=2)
    _, s_one = ctx.sigma(field[-1:], dirs[-1:], c0d[-1:].contiguous(), cd[-1:].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(s_one[0], s_mfma[-1])  # a batch and one of its RHS alone: the same sums
    _, got = gpu_lib.from_planes(torch.zeros_like(c0d), s_mfma)
    _, val = gpu_lib.from_planes(torch.zeros_like(c0d), s_valu)
    tol = 5e-6 if precision == "fp32" else 2e-5
    worst = 0.0
    for r in range(0, nrhs, max(1, nrhs // 6)):
        ref = O.apply_H(op, O.dipole_blocks(op, dirs[r]), field[r], c0[r], c[r])[1]
        scale = np.max(np.abs(ref))
        worst = max(worst, np.max(np.abs(got[r] - ref)) / scale)
        assert np.max(np.abs(val[r] - ref)) / scale < tol
    say(f"[coulomb mfma] o={o} v={v} N_Q={nq} {nrhs} RHS {precision}: sigma rel err {worst:.2e}")
    assert worst < tol
