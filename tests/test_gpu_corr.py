"""Time-correlation output R(t) = <X(0+) | X(t)> (eq. time_correlation_function) of
rttda_propagate and rttda_propagate_sso against the FP64 oracle.

R(t) is dominated by the ground amplitude (|c0|^2 ~ 1, constant without a field); the excited
part is O(kappa^2).  The bar is the trace bar applied to the excited part: |R_gpu - R_oracle|
<= 1e-5 (FP32) / 1e-4 (mixed) times max |R - conj(c0ref) c0|."""
import numpy as np
import pytest

from conftest import say
from oracle import rttda64 as O
from paper_2601_16949_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "mixed": 1e-4}


@pytest.mark.parametrize("prec,integrator", [("fp32", "rk4"), ("fp32", "sso"), ("mixed", "rk4"), ("mixed", "sso")])
def test_correlation_matches_oracle(gpu_lib, prec, integrator):
    import torch
    from paper_2601_16949_amd import rttda

    o, v, nq, n = 10, 40, 120, 300
    shape = I.Shape(o, v, nq, b_scale=0.05, storage="f32" if prec == "fp32" else "bf16")
    prob = I.make_problem(shape, 4711)
    op = O.Operator.from_problem(prob)
    ctx = rttda.Context(rttda.DeviceProblem(prob, prec), max_rhs=2)
    pulses = I.kick_pulses(axes=[(0.0, 0.0, 1.0), (0.6, 0.8, 0.0)], kappa=0.02)
    c0d, cd = gpu_lib.ground_state(2, o, v)
    corr = torch.full((n + 1, 2, 2), float("nan"), dtype=torch.float64, device="cuda")
    ctx.propagate(pulses, 0.05, n, c0d, cd, corr=corr, integrator=integrator)
    torch.cuda.synchronize()
    got = corr.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    assert np.isfinite(got).all()
    for r, p in enumerate(pulses):
        ref = O.propagate_correlation(op, p, 0.05, n, integrator)
        blocks = O.dipole_blocks(op, p.direction)
        c0k, _ = O.kick(blocks, p.e0, 1.0 + 0j, np.zeros((o, v), complex))
        exc = ref - abs(c0k) ** 2  # without a field c0 stays at its kicked value
        err = np.max(np.abs(got[:, r] - ref))
        say(f"[corr] {prec} {integrator} rhs {r}: max |R_gpu - R_ora| = {err:.2e}, max |R_exc| = {np.max(np.abs(exc)):.2e}")
        assert abs(got[0, r].imag) < 1e-15 and abs(got[0, r].real - O.norm2(*O.kick(blocks, p.e0, 1.0 + 0j, np.zeros((o, v), complex)))) < 1e-12
        assert err <= TOL[prec] * np.max(np.abs(exc))


def test_correlation_applies_to_one_call(gpu_lib):
    """The output is consumed by the next call: a second call without it leaves the array alone,
    and the graph replay with and without it gives the same trace."""
    import torch
    from paper_2601_16949_amd import rttda

    o, v, nq, n = 8, 24, 30, 40
    prob = I.make_problem(I.Shape(o, v, nq, b_scale=0.05, storage="f32"), 99)
    ctx = rttda.Context(rttda.DeviceProblem(prob, "fp32"), max_rhs=1)
    pulses = I.kick_pulses(axes=[(0.0, 0.0, 1.0)], kappa=0.01)
    c0a, ca = gpu_lib.ground_state(1, o, v)
    corr = torch.zeros((n + 1, 1, 2), dtype=torch.float64, device="cuda")
    ta = ctx.propagate(pulses, 0.05, n, c0a, ca, corr=corr)
    torch.cuda.synchronize()
    first = corr.clone()
    c0b, cb = gpu_lib.ground_state(1, o, v)
    tb = ctx.propagate(pulses, 0.05, n, c0b, cb)
    torch.cuda.synchronize()
    assert torch.equal(first, corr)
    assert torch.equal(ta, tb) and torch.equal(ca, cb)
    # a call refused by the binding (65 population vectors, above the limit of 64) leaves no
    # correlation output pending for the call after it
    bad_u = torch.zeros((65, o, v), dtype=torch.float64, device="cuda")
    bad_p = torch.zeros((n + 1, 1, 65), dtype=torch.float64, device="cuda")
    c0c, cc = gpu_lib.ground_state(1, o, v)
    with pytest.raises(gpu_lib.RttdaError):
        ctx.propagate(pulses, 0.05, n, c0c, cc, corr=corr, pops=bad_p, pop_vectors=bad_u)
    c0d, cd = gpu_lib.ground_state(1, o, v)
    ctx.propagate(pulses, 0.05, n, c0d, cd)
    torch.cuda.synchronize()
    assert torch.equal(first, corr)
    assert torch.equal(c0c, gpu_lib.ground_state(1, o, v)[0]) and torch.equal(cd, cb)
