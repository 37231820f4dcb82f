"""Full-length runs of the large workloads against the FP64 oracle's cached references
(tests/golden/make_long_traces.py, which calls only the oracle and the input generator):

* o60 v400 N_Q1500, x/y/z kicks, 20000 RK4 steps, in FP32 (dipole trace within 1e-5) and in split
  BF16 (within 1e-4; spectral peaks within 1e-4 Ha), in the launch configuration bench.py times;
  the same 20000 steps through the split operator;
* o40 v300 N_Q1000, Gaussian-envelope cosine pulses at four carriers of the 64-carrier scan and
  E0 = 0.01 and 0.05 (resonant Rabi cycling and the two-photon carrier), 16000 steps: traces within
  1e-5 and the populations of the ground state and the 8 lowest TI-TDA states within 1e-5;
* o240 v1800 N_Q5000 (BF16 factors), x/y/z kicks: the z trace of the first steps within 1e-4.
"""
import os

import numpy as np
import pytest
from conftest import say

from oracle import spectrum as SP
from paper_2601_16949_amd import inputs as I

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    return np.load(os.path.join(GOLDEN, name), allow_pickle=False)


def _run_in_parts(ctx, pulses, dt, n, c0, c, parts=4, **kw):
    """Propagate n steps as `parts` consecutive calls (a progress line after each), trace joined."""
    import torch

    out = torch.empty((n + 1, len(pulses)), dtype=torch.float64, device="cuda")
    done = 0
    for k in range(parts):
        m = (n - done) // (parts - k)
        tr = ctx.propagate(pulses, dt, m, c0, c, step0=done, **kw)
        out[done:done + m + 1] = tr
        done += m
        torch.cuda.synchronize()
        say(f"   {done}/{n} steps")
    return out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,tol,peak_tol", [("fp32", 1e-5, 1e-5), ("mixed", 1e-4, 1e-4)])
def test_o60_v400_full_trace(gpu_lib, precision, tol, peak_tol):
    import torch

    g = _load(f"cfg2_trace_{precision}.npz")
    ref = g["trace"]
    wl = I.workload(2)
    shape = I.Shape(wl.shape.o, wl.shape.v, wl.shape.nq, wl.shape.b_scale, storage="f32" if precision == "fp32" else "bf16")
    prob = I.make_problem(shape, wl.seed)
    ctx = gpu_lib.Context(gpu_lib.DeviceProblem(prob, precision), max_rhs=3)
    tuned = ctx.use_tuned(3)
    say(f"[o60 v400 {precision}] {wl.n_steps} steps, 3 RHS, autotuned {tuned}")
    c0, c = gpu_lib.ground_state(3, shape.o, shape.v)
    got = _run_in_parts(ctx, wl.pulses, wl.dt, wl.n_steps, c0, c).cpu().numpy()
    assert ctx.guard() == -1
    for r in range(3):
        err = np.max(np.abs(got[:, r] - ref[:, r])) / np.max(np.abs(ref[:, r]))
        pg = SP.peaks(got[:, r], wl.dt, I.KAPPA, omega_max=3.0)
        po = SP.peaks(ref[:, r], wl.dt, I.KAPPA, omega_max=3.0)
        dw = max(abs(a - b) for (a, _), (b, _) in zip(pg, po)) if len(pg) == len(po) else float("inf")
        say(f"   direction {r}: trace rel err {err:.2e}, {len(po)} peaks, max shift {dw:.2e} Ha")
        assert err < tol
        assert len(pg) == len(po) and dw < peak_tol


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,tol,peak_tol", [("fp32", 1e-5, 1e-5), ("mixed", 1e-4, 1e-4)])
def test_o60_v400_full_trace_split_operator(gpu_lib, precision, tol, peak_tol):
    """The paper's split operator over the same 20000 steps against the oracle's eigen route of the
    split operator's mode map."""
    g = _load(f"cfg2_trace_sso_{precision}.npz")
    ref = g["trace"]
    wl = I.workload(2)
    shape = I.Shape(wl.shape.o, wl.shape.v, wl.shape.nq, wl.shape.b_scale, storage="f32" if precision == "fp32" else "bf16")
    prob = I.make_problem(shape, wl.seed)
    ctx = gpu_lib.Context(gpu_lib.DeviceProblem(prob, precision), max_rhs=3)
    tuned = ctx.use_tuned(3, "sso")
    say(f"[o60 v400 {precision} split operator] {wl.n_steps} steps, 3 RHS, autotuned {tuned}")
    c0, c = gpu_lib.ground_state(3, shape.o, shape.v)
    got = _run_in_parts(ctx, wl.pulses, wl.dt, wl.n_steps, c0, c, integrator="sso").cpu().numpy()
    assert ctx.guard() == -1
    for r in range(3):
        err = np.max(np.abs(got[:, r] - ref[:, r])) / np.max(np.abs(ref[:, r]))
        pg = SP.peaks(got[:, r], wl.dt, I.KAPPA, omega_max=3.0)
        po = SP.peaks(ref[:, r], wl.dt, I.KAPPA, omega_max=3.0)
        dw = max(abs(a - b) for (a, _), (b, _) in zip(pg, po)) if len(pg) == len(po) else float("inf")
        say(f"   direction {r}: trace rel err {err:.2e}, {len(po)} peaks, max shift {dw:.2e} Ha")
        assert err < tol
        assert len(pg) == len(po) and dw < peak_tol


@pytest.mark.timeout(600)
def test_o40_v300_rabi_populations(gpu_lib):
    import torch

    g = _load("cfg4_rabi_populations.npz")
    wl = I.workload(4)
    prob = I.make_problem(wl.shape, wl.seed)
    pulses = [I.Pulse(kind=I.PULSE_GAUSS, e0=float(e0), omega=float(w), t0=400.0, fwhm=400.0, phase=np.pi / 2,
                      direction=(0.0, 0.0, 1.0)) for e0, w in zip(g["e0"], g["omega"])]
    R, n, every = len(pulses), wl.n_steps, int(g["pop_every"])
    ctx = gpu_lib.Context(gpu_lib.DeviceProblem(prob, "fp32"), max_rhs=R)
    U = torch.from_numpy(np.ascontiguousarray(g["evecs"])).cuda()
    c0, c = gpu_lib.ground_state(R, wl.shape.o, wl.shape.v)
    say(f"[o40 v300] {R} pulses (E0 {sorted(set(g['e0'].tolist()))}), {n} steps, populations of 8 states")
    tr, pops = np.empty((n + 1, R)), np.empty((n + 1, R, U.shape[0]))
    done = 0
    for part in range(4):  # four consecutive calls, a progress line after each
        m = (n - done) // (4 - part)
        pp = torch.empty((m + 1, R, U.shape[0]), dtype=torch.float64, device="cuda")
        t = ctx.propagate(pulses, wl.dt, m, c0, c, step0=done, pops=pp, pop_vectors=U)
        torch.cuda.synchronize()
        tr[done:done + m + 1], pops[done:done + m + 1] = t.cpu().numpy(), pp.cpu().numpy()
        done += m
        say(f"   {done}/{n} steps")
    assert ctx.guard() == -1
    ref_tr, ref_pops = g["trace"], g["pops"]
    err_tr = np.max(np.abs(tr - ref_tr), axis=0) / np.max(np.abs(ref_tr), axis=0)
    got_p = pops[::every]
    err_p = np.max(np.abs(got_p - ref_pops[:, :, 1:]))
    say(f"   trace rel err per pulse {np.array2string(err_tr, precision=2)}; populations max abs err {err_p:.2e}; "
        f"largest excited population {ref_pops[:, :, 1:].max():.3f}")
    assert np.all(err_tr < 1e-5)
    assert err_p < 1e-5
    assert ref_pops[:, :, 1:].max() > 0.01  # the pulses move population into the lowest states


@pytest.mark.timeout(900)
def test_o240_v1800_first_steps(gpu_lib):
    """o240 v1800 N_Q5000 with BF16 factors drawn on the host exactly as the oracle's reference
    read them (streamed to the device in Q ranges): the z-kick trace of the first steps of the
    batched x/y/z run against the oracle's direct route."""
    import torch

    g = _load("cfg3_trace_z.npz")
    ref = g["trace"]
    n = ref.size - 1
    wl = I.workload(3)
    say(f"[o240 v1800 N_Q5000] drawing the BF16 factors on the host ({wl.shape.nq} Q), {n} reference steps")
    t = I.upload_factors_streamed(wl.shape, wl.seed, threads=16,
                                  progress=lambda q: say(f"   {q} Q uploaded") if q % 640 == 0 or q == wl.shape.nq else None)
    ctx = gpu_lib.Context(gpu_lib.DeviceProblem.from_tensors(wl.shape, t, "mixed"), max_rhs=3)
    ctx.use_tuned(3)
    c0, c = gpu_lib.ground_state(3, wl.shape.o, wl.shape.v)
    tr = ctx.propagate(wl.pulses, wl.dt, n, c0, c)
    torch.cuda.synchronize()
    got = tr.cpu().numpy()[:, 2]
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say(f"   z trace over {n} steps: rel err {err:.2e}")
    assert ctx.guard() == -1
    assert err < 1e-4
