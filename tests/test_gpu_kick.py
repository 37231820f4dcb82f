"""Unitary delta kick (RTTDA_PULSE_DELTA_EXACT: X <- exp(i kappa M) X) on the device against the
oracle's matrix exponential of the dense CSF dipole, alone and batched with a first-order kick,
followed by RK4 / split-operator propagation (trace bar 1e-5 relative in FP32)."""
import numpy as np
import pytest

from conftest import say
from oracle import rttda64 as O
from paper_2601_16949_amd import inputs as I

pytestmark = pytest.mark.gpu


def _ctx(o, v, nq, seed, max_rhs):
    from paper_2601_16949_amd import rttda

    prob = I.make_problem(I.Shape(o, v, nq, b_scale=0.05, storage="f32"), seed)
    return O.Operator.from_problem(prob), rttda.Context(rttda.DeviceProblem(prob, "fp32"), max_rhs=max_rhs)


@pytest.mark.parametrize("integrator", ["rk4", "sso"])
def test_exact_kick_state_and_trace(gpu_lib, integrator):
    import torch

    o, v, nq, n = 10, 40, 120, 200
    op, ctx = _ctx(o, v, nq, 2468, 2)
    pulses = [I.Pulse(kind=I.PULSE_DELTA_EXACT, e0=0.3, direction=(0.0, 0.0, 1.0)),
              I.Pulse(kind=I.PULSE_DELTA, e0=0.01, direction=(0.6, 0.0, 0.8))]
    # the kicked state alone (no steps)
    c0d, cd = gpu_lib.ground_state(2, o, v)
    ctx.propagate(pulses, 0.05, 0, c0d, cd, want_trace=False, integrator=integrator)
    torch.cuda.synchronize()
    g0, G = gpu_lib.from_planes(c0d, cd)
    for r, p in enumerate(pulses):
        blocks = O.dipole_blocks(op, p.direction)
        e0, E = O.apply_kick(op, blocks, p, 1.0 + 0j, np.zeros((o, v), complex))
        err = max(abs(g0[r] - e0), np.max(np.abs(G[r] - E)))
        say(f"[exact kick] {integrator} rhs {r} kind {p.kind}: max |X_gpu - X_ora| = {err:.2e}, |X|^2 = {O.norm2(e0, E):.15f}")
        assert err < 1e-12
    # trace after the kick
    c0d, cd = gpu_lib.ground_state(2, o, v)
    tr = ctx.propagate(pulses, 0.05, n, c0d, cd, integrator=integrator).cpu().numpy()
    for r, p in enumerate(pulses):
        prop = O.propagate if integrator == "rk4" else O.propagate_sso
        ref = prop(op, p, 0.05, n)[0]
        rel = np.max(np.abs(tr[:, r] - ref)) / np.max(np.abs(ref))
        say(f"[exact kick] {integrator} rhs {r}: trace rel err {rel:.2e}")
        assert rel < 1e-5


def test_exact_kick_rejects_too_strong_a_kick(gpu_lib):
    o, v, nq = 6, 20, 10
    _, ctx = _ctx(o, v, nq, 11, 1)
    c0d, cd = gpu_lib.ground_state(1, o, v)
    with pytest.raises(gpu_lib.RttdaError):
        ctx.propagate([I.Pulse(kind=I.PULSE_DELTA_EXACT, e0=500.0, direction=(0.0, 0.0, 1.0))], 0.05, 1, c0d, cd)
