"""rttda_sigma_noalloc (the static-scratch sigma for callers that cannot allocate) against rttda_sigma
on the same inputs, to the sigma parity bars; two calls in a row, the second with a smaller input."""
import numpy as np
import pytest
from conftest import say

from paper_2601_16949_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"fp32": 5e-6, "mixed": 2e-5}


def _case(gpu_lib, o, v, nq, nrhs, precision, seed):
    import torch

    storage = "f32" if precision == "fp32" else "bf16"
    prob = I.make_problem(I.Shape(o, v, nq, 0.05, storage=storage), seed)
    dev = gpu_lib.DeviceProblem(prob, precision)
    c0h, ch = I.random_state(o, v, nrhs, seed + 1)
    c0, c = gpu_lib.to_planes(c0h, ch)
    field = [0.01 * (r + 1) for r in range(nrhs)]
    dirs = [I.AXES[r % 3] for r in range(nrhs)]
    ctx = gpu_lib.Context(dev, max_rhs=nrhs)
    ref0, ref = ctx.sigma(field, dirs, c0, c)
    got0, got = gpu_lib.sigma_noalloc(dev, field, dirs, c0, c)
    torch.cuda.synchronize()
    scale = float(torch.max(torch.abs(ref)))
    err = float(torch.max(torch.abs(got - ref))) / scale
    err0 = float(torch.max(torch.abs(got0 - ref0))) / max(float(torch.max(torch.abs(ref0))), 1e-300)
    same = bool(torch.equal(got, ref) and torch.equal(got0, ref0))
    say(f"   o={o} v={v} N_Q={nq} nrhs={nrhs} {precision}: rel err {err:.2e} (s0 {err0:.2e}), bitwise {same}")
    assert err <= TOL[precision] and err0 <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_sigma_noalloc_matches_sigma_twice(gpu_lib, precision):
    say(f"[sigma_noalloc] {precision}")
    _case(gpu_lib, 60, 400, 300, 3, precision, 21)  # more Q splits than the static slabs hold
    _case(gpu_lib, 10, 40, 120, 1, precision, 22)   # the second call: a smaller input


def test_sigma_noalloc_refuses_what_does_not_fit(gpu_lib):
    import torch

    prob = I.make_problem(I.Shape(4, 8, 3), 5)
    dev = gpu_lib.DeviceProblem(prob, "fp32")
    c0, c = gpu_lib.ground_state(1, 4, 8)
    with pytest.raises(gpu_lib.RttdaError) as ex:
        gpu_lib.sigma_noalloc(dev, [0.0] * 65, [I.AXES[2]] * 65, torch.zeros((65, 2), dtype=torch.float64,
                                                                              device="cuda"),
                              torch.zeros((65, 2, 4, 8), dtype=torch.float64, device="cuda"))
    assert ex.value.status == gpu_lib.E_INVAL
    big = gpu_lib.DeviceProblem.__new__(gpu_lib.DeviceProblem)
    big.o, big.v, big.nq, big.cx, big.precision = 240, 1800, 8, 0.2, "fp32"
    big.e_occ, big.e_virt, big.mu = dev.e_occ, dev.e_virt, dev.mu
    big.b_ov = big.b_oo = big.b_vv = dev.b_ov
    c0b = torch.zeros((3, 2), dtype=torch.float64, device="cuda")
    cb = torch.zeros((3, 2, 240, 1800), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.RttdaError) as ex:
        gpu_lib.sigma_noalloc(big, [0.0] * 3, [I.AXES[2]] * 3, c0b, cb)
    assert ex.value.status == gpu_lib.E_NOMEM
