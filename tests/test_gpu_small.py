"""The small-problem path (one launch for a stage's Coulomb and exchange partial sums, one
single-workgroup launch for the whole stage epilogue) against the FP64 oracle and against the
general kernels: RK4 with a kick and a pulse, in FP32 and split BF16, the split operator on the
same slabs, graph replay against direct launches, and two launches per RK4 stage."""
import numpy as np
import pytest
from conftest import say

from oracle import rttda64 as O
from paper_2601_16949_amd import inputs as I

pytestmark = pytest.mark.gpu


def _pulses():
    return [I.Pulse(kind=I.PULSE_DELTA, e0=1e-3, direction=(0.0, 0.0, 1.0)),
            I.Pulse(kind=I.PULSE_GAUSS, e0=0.04, omega=0.6, t0=3.0, fwhm=3.0, direction=(1.0, 0.0, 0.0)),
            I.Pulse(kind=I.PULSE_CHIRP, e0=0.03, omega=0.5, t0=2.0, fwhm=4.0, beta=0.02, phase=0.3,
                    direction=(0.0, 0.6, 0.8))]


@pytest.mark.parametrize("o,v,nq,precision,integrator", [(10, 40, 120, "fp32", "rk4"), (10, 40, 120, "mixed", "rk4"),
                                                        (13, 37, 20, "fp32", "rk4"), (32, 64, 50, "mixed", "rk4"),
                                                        (10, 40, 120, "fp32", "sso"), (7, 9, 3, "mixed", "sso")])
def test_small_path_matches_oracle_and_general_kernels(gpu_lib, o, v, nq, precision, integrator):
    import torch

    storage = "f32" if precision == "fp32" else "bf16"
    prob = I.make_problem(I.Shape(o, v, nq, 0.05, storage=storage), 900 + o)
    op = O.Operator.from_problem(prob)
    pulses = _pulses()
    dt, n = 0.05, 120
    ctx = gpu_lib.Context(gpu_lib.DeviceProblem(prob, precision), max_rhs=3)
    # the default: the small path only where the exchange has at most 2e7 flops per stage
    small_default = 4.0 * nq * o * v * (o + v) * 3 <= 2e7 and o * v <= 2048
    assert ctx.get_tuning()["small_path"] == (1 if small_default else 2)
    out = {}
    for mode in (1, 2):
        ctx.set_tuning(small_path=mode)
        c0, c = gpu_lib.ground_state(3, o, v)
        out[mode] = ctx.propagate(pulses, dt, n, c0, c, integrator=integrator).cpu().numpy()
    tol = 1e-5 if precision == "fp32" else 1e-4
    route = O.propagate if integrator == "rk4" else O.propagate_sso
    worst = 0.0
    for r, p in enumerate(pulses):
        ref, _, _ = route(op, p, dt, n)
        scale = np.max(np.abs(ref))
        e_small = np.max(np.abs(out[1][:, r] - ref)) / scale
        e_gen = np.max(np.abs(out[2][:, r] - ref)) / scale
        worst = max(worst, e_small)
        assert e_small < tol and e_gen < tol, (r, e_small, e_gen)
    say(f"[small path] o={o} v={v} N_Q={nq} {precision} {integrator}: worst trace rel err {worst:.2e}")


def test_small_path_graph_equals_direct_and_launch_count(gpu_lib):
    import torch

    prob = I.make_problem(I.Shape(10, 40, 120, 0.05), I.SEED_BASE + 1)
    ctx = gpu_lib.Context(gpu_lib.DeviceProblem(prob, "fp32"), max_rhs=3)
    pulses = _pulses()
    res = {}
    for mode in (1, 2):  # graph replay, direct launches
        ctx.set_tuning(use_graph=mode, steps_per_graph=8, small_path=1)
        c0, c = gpu_lib.ground_state(3, 10, 40)
        res[mode] = (ctx.propagate(pulses, 0.05, 64, c0, c), c)
    assert torch.equal(res[1][0], res[2][0]) and torch.equal(res[1][1], res[2][1])
    # two launches per RK4 stage: the partial sums ("exchange" class) and the stage epilogue
    ctx.set_profiling(True)
    c0, c = gpu_lib.ground_state(3, 10, 40)
    ctx.propagate(pulses, 0.05, 10, c0, c)
    prof = ctx.get_profile()
    ctx.set_profiling(False)
    say(f"[small path] launches over 10 steps: {prof}")
    assert prof["exchange"]["launches"] == 40 and prof["epilogue"]["launches"] == 40
    assert prof["coulomb"]["launches"] == 0
