"""Serving loop on the GPU: each request's trace is the same alone and in a mix (bitwise, the
kernels use no atomics), admission respects the HBM budget, and a probe request matches the
FP64 oracle (mixed-precision tolerance 1e-4)."""
import sys

import numpy as np
import pytest
from conftest import say

from oracle import rttda64 as O
from paper_2601_16949_amd import inputs as I

pytestmark = pytest.mark.gpu




def small_requests(n, seed=11, o_max=24):
    reqs = I.serving_requests(n, rate=200.0, seed=seed, o_min=4, o_max=o_max)
    for r in reqs:
        r.n_steps = 60 + (r.rid * 37) % 90
        if r.pulse.kind == I.PULSE_GAUSS:
            r.pulse.t0 = 0.5 * r.n_steps * r.dt
            r.pulse.fwhm = 2.0
    return reqs


def test_alone_equals_mix_and_budget(gpu_lib):
    from paper_2601_16949_amd import serve

    reqs = small_requests(8)
    say("[serving] mix of 8")
    srv = serve.Server(budget_bytes=2 << 30, chunk_steps=32, precision="mixed")
    stats = srv.run(reqs, realtime=False)
    say(f"   {stats}")
    assert stats["max_concurrent"] >= 2
    mix = {r.rid: srv.results[r.rid].trace for r in reqs}
    for r in reqs[:3]:
        alone = serve.Server(budget_bytes=2 << 30, chunk_steps=32, precision="mixed")
        alone.run([r], realtime=False)
        assert np.array_equal(alone.results[r.rid].trace, mix[r.rid]), r.rid
    # a budget that fits only the largest request alone forces one-at-a-time service
    big = max(serve.footprint(r.shape, r.n_steps, "mixed") for r in reqs)
    tight = serve.Server(budget_bytes=big, chunk_steps=32, precision="mixed")
    st2 = tight.run(reqs, realtime=False)
    assert tight.peak_used <= big
    for r in reqs:
        assert np.array_equal(tight.results[r.rid].trace, mix[r.rid])
    say(f"   tight budget: max_concurrent {st2['max_concurrent']}")


def test_unstable_request_is_refused(gpu_lib):
    """A request whose time step exceeds the RK4 stability limit for its operator is refused at
    admission (it takes no slot and no memory); the other requests are served as without it."""
    from paper_2601_16949_amd import serve

    reqs = small_requests(4, seed=13)
    say("[serving] unstable request in a mix of 4")
    base = serve.Server(budget_bytes=1 << 30, chunk_steps=32, precision="mixed")
    base.run(reqs, realtime=False)
    bad = reqs[2]
    bad.dt = 40.0  # rho(A) is at least the lowest excitation (above 0.1 Ha here): rho dt > 4
    srv = serve.Server(budget_bytes=1 << 30, chunk_steps=32, precision="mixed")
    st = srv.run(reqs, realtime=False)
    say(f"   {st['refused']} refused: {srv.results[bad.rid].refused}")
    assert st["refused"] == 1 and srv.results[bad.rid].refused
    assert srv.results[bad.rid].trace is None and srv.peak_used <= base.peak_used
    for r in reqs:
        if r is not bad:
            assert not srv.results[r.rid].refused
            assert np.array_equal(srv.results[r.rid].trace, base.results[r.rid].trace), r.rid


def test_probe_request_matches_oracle(gpu_lib):
    import torch
    from paper_2601_16949_amd import serve

    r = small_requests(3, seed=5, o_max=12)[0]
    r.pulse = I.Pulse(kind=I.PULSE_GAUSS, e0=0.02, omega=0.5, t0=3.0, fwhm=2.0, direction=(0, 0, 1))
    say(f"[serving probe] o={r.shape.o} v={r.shape.v} nq={r.shape.nq} steps={r.n_steps}")
    srv = serve.Server(budget_bytes=1 << 30, chunk_steps=40, precision="mixed")
    srv.run([r], realtime=False)
    got = srv.results[r.rid].trace
    t = I.make_device_tensors(r.shape, r.seed)
    prob = I.problem_from_device(r.shape, r.seed, t)
    ref, _, _ = O.propagate(O.Operator.from_problem(prob), r.pulse, r.dt, r.n_steps)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say(f"   trace rel err {err:.2e}")
    assert err < 1e-4


@pytest.mark.parametrize("integrator", ["rk4", "sso"])
def test_pool_api_budget_chunks_and_release(gpu_lib, integrator):
    """The library pool: admission beyond the budget is refused (E_NOMEM); a request stepped in
    chunks through the pool gives bitwise the trace and state of one direct propagate call; the
    budget returns on release."""
    import torch
    from paper_2601_16949_amd import rttda

    o, v = 12, 30
    prob = I.make_problem(I.Shape(o, v, 24), 3)
    dev = rttda.DeviceProblem(prob, "fp32")
    pulses = [I.Pulse(kind=I.PULSE_GAUSS, e0=0.03, omega=0.5, t0=2.0, fwhm=2.0, direction=(0, 0, 1)),
              I.Pulse(kind=I.PULSE_DELTA, e0=1e-3, direction=(1, 0, 0))]
    n = 137
    say(f"[pool] {integrator}")
    ctx_a, ctx_b = rttda.Context(dev, 2), rttda.Context(dev, 2)
    c0a, ca = gpu_lib.ground_state(2, o, v)
    c0b, cb = gpu_lib.ground_state(2, o, v)
    direct = ctx_a.propagate(pulses, 0.05, n, c0a, ca, integrator=integrator)
    pool = rttda.Pool(1000)
    trace = torch.empty((n + 1, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(rttda.RttdaError):
        pool.admit(ctx_b, pulses, 0.05, n, c0b, cb, trace, footprint=2000, integrator=integrator)
    slot = pool.admit(ctx_b, pulses, 0.05, n, c0b, cb, trace, footprint=600, integrator=integrator)
    assert pool.usage() == (600, 1)
    chunks = 0
    while not pool.poll(slot)[1]:
        chunks += pool.step(40)
    assert chunks == 4 and pool.poll(slot)[0] == n
    pool.release(slot)
    assert pool.usage() == (0, 0)
    torch.cuda.synchronize()
    assert torch.equal(trace, direct)
    assert torch.equal(cb, ca) and torch.equal(c0b, c0a)
    pool.close()
