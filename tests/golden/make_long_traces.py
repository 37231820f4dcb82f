"""Writes the oracle's long-run references for the GPU parity tests of the full-size workloads.
Calls only the FP64 oracle and the seeded input generator (the inputs are the stored values the
GPU path reads: FP32- or BF16-rounded factors).

    python tests/golden/make_long_traces.py cfg2 fp32|mixed
        o60 v400 N_Q1500, x/y/z first-order kicks (kappa 1e-4), dt 0.05, 20000 RK4 steps: the full
        dipole trace of each direction from the eigen route (dense A, eigh, exact field-free RK4
        map, the trace evaluated in the amplitude basis) -> cfg2_trace_<precision>.npz
    python tests/golden/make_long_traces.py cfg4
        o40 v300 N_Q1000, Gaussian-envelope cosine pulses along z (FWHM 400 au, t0 400 au) at the
        carriers 0.5, 0.7, 1.0 and 1.2 times the lowest excitation energy (scan indices 0, 18, 45
        and 63 of the 64-carrier scan) and E0 = 0.01 and 0.05, dt 0.05, 16000 RK4 steps in the
        eigenbasis: traces, and the populations of the ground state and of the 8 lowest TI-TDA
        states every 8 steps, plus those 8 eigenvectors -> cfg4_rabi_populations.npz
    python tests/golden/make_long_traces.py cfg2sso fp32|mixed
        the same shape and kicks through the split operator (eigen route of its mode map) ->
        cfg2_trace_sso_<precision>.npz
    python tests/golden/make_long_traces.py cfg3 N [OUT]
        o240 v1800 N_Q5000 (BF16 factors), z first-order kick, dt 0.1: the first N RK4 steps of
        the direct density-fitted route with the factors read per Q range -> cfg3_trace_z.npz
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import rttda64 as O  # noqa: E402
from paper_2601_16949_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
T0 = time.time()


def say(msg):
    print(f"[{time.time() - T0:7.0f} s] {msg}", flush=True)


def cfg2(precision):
    wl = I.workload(2)
    shape = I.Shape(wl.shape.o, wl.shape.v, wl.shape.nq, wl.shape.b_scale,
                    storage="f32" if precision == "fp32" else "bf16")
    op = O.Operator.from_problem(I.make_problem(shape, wl.seed))
    say(f"cfg2 {precision}: dense A and eigh at n = {op.o * op.v}")
    route = O.EigenRoute(op)
    say(f"eigh done: lowest {route.w[1]:.12f} Ha, highest {route.w[-1]:.12f} Ha")
    trace = np.empty((wl.n_steps + 1, len(wl.pulses)))
    for r, p in enumerate(wl.pulses):
        trace[:, r] = route.field_free_trace_blocked(p, wl.dt, wl.n_steps)
        say(f"direction {r} done")
    np.savez(os.path.join(HERE, f"cfg2_trace_{precision}.npz"), trace=trace, dt=wl.dt, kappa=I.KAPPA,
             w_lowest=route.w[1], w_highest=route.w[-1],
             note=np.array(f"{wl.name} {precision}: oracle eigen route, full dipole trace per direction (x, y, z)"))


def cfg2_sso(precision):
    wl = I.workload(2)
    shape = I.Shape(wl.shape.o, wl.shape.v, wl.shape.nq, wl.shape.b_scale,
                    storage="f32" if precision == "fp32" else "bf16")
    op = O.Operator.from_problem(I.make_problem(shape, wl.seed))
    say(f"cfg2 split operator {precision}: dense A and eigh at n = {op.o * op.v}")
    route = O.EigenRoute(op)
    say(f"eigh done: lowest {route.w[1]:.12f} Ha, highest {route.w[-1]:.12f} Ha")
    trace = np.empty((wl.n_steps + 1, len(wl.pulses)))
    for r, p in enumerate(wl.pulses):
        trace[:, r] = route.field_free_trace_sso_blocked(p, wl.dt, wl.n_steps)
        say(f"direction {r} done")
    np.savez(os.path.join(HERE, f"cfg2_trace_sso_{precision}.npz"), trace=trace, dt=wl.dt, kappa=I.KAPPA,
             w_lowest=route.w[1], w_highest=route.w[-1],
             note=np.array(f"{wl.name} {precision}: oracle eigen route of the split operator, full dipole trace "
                           f"per direction (x, y, z)"))


CFG4_SCAN = (0, 18, 45, 63)
CFG4_E0 = (0.01, 0.05)


def cfg4_pulses(w1):
    out = []
    for e0 in CFG4_E0:
        scan = I.gauss_cos_scan(w1, e0)
        out += [scan[k] for k in CFG4_SCAN]
    return out


def cfg4():
    wl = I.workload(4)
    op = O.Operator.from_problem(I.make_problem(wl.shape, wl.seed))
    say(f"cfg4: dense A and eigh at n = {op.o * op.v}")
    route = O.EigenRoute(op)
    w1 = float(route.w[1])
    say(f"eigh done: lowest excitation {w1:.12f} Ha")
    pulses = cfg4_pulses(w1)
    trace, pops = route.propagate_rk4_many(pulses, wl.dt, wl.n_steps, n_pop=8, pop_every=8,
                                           progress=lambda n: say(f"step {n}"))
    np.savez(os.path.join(HERE, "cfg4_rabi_populations.npz"), trace=trace, pops=pops, pop_every=8,
             evecs=np.ascontiguousarray(route.U[1:, 1:9].T.reshape(8, op.o, op.v)), w=route.w[1:9],
             omega=np.array([p.omega for p in pulses]), e0=np.array([p.e0 for p in pulses]), dt=wl.dt,
             note=np.array(f"{wl.name}: oracle eigenbasis RK4 with the field, scan indices {CFG4_SCAN} "
                           f"at E0 {CFG4_E0}; pops[:, r, 0] = |c0|^2, pops[:, r, 1:] = eigenstates 1..8"))


def cfg3(n_steps, out=None):
    import concurrent.futures as cf

    wl = I.workload(3)
    shape = wl.shape
    say(f"cfg3: drawing the BF16 factors ({shape.nq} Q)")
    o, v, nq = shape.o, shape.v, shape.nq
    bits = (np.empty((nq, o, v), np.uint16), np.empty((nq, o, o), np.uint16), np.empty((nq, v, v), np.uint16))
    with cf.ThreadPoolExecutor(max_workers=8) as pool:
        for q0 in range(0, nq, 250):
            q1 = min(nq, q0 + 250)
            part = I.factor_bits_range(shape, wl.seed, q0, q1, pool)
            for dst, src in zip(bits, part):
                dst[q0:q1] = src
    e_occ, e_virt = I.gen_energies(shape, wl.seed)
    op = O.Operator(e_occ, e_virt, O.BF16Stored(bits[0]), O.BF16Stored(bits[1]), O.BF16Stored(bits[2]),
                    I.gen_mu(shape, wl.seed), shape.cx)
    say("factors drawn")
    p = wl.pulses[2]  # z kick
    blocks = O.dipole_blocks(op, p.direction)
    c0, C = O.apply_kick(op, blocks, p, 1.0 + 0j, np.zeros((o, v), dtype=np.complex128))
    trace = [O.dipole_expectation(blocks, c0, C)]
    norms = [O.norm2(c0, C)]
    for n in range(n_steps):
        c0, C = O.rk4_step(op, blocks, p, wl.dt, n, c0, C)
        trace.append(O.dipole_expectation(blocks, c0, C))
        norms.append(O.norm2(c0, C))
        say(f"step {n + 1}: trace {trace[-1]:.15e}")
        np.savez(out or os.path.join(HERE, "cfg3_trace_z.npz"), trace=np.array(trace), norms=np.array(norms), dt=wl.dt,
                 kappa=p.e0, note=np.array(f"{wl.name}: oracle direct DF route (FP64, BF16-stored factors), z kick, "
                                           f"first {n + 1} RK4 steps"))


if __name__ == "__main__":
    which = sys.argv[1]
    if which == "cfg2":
        cfg2(sys.argv[2])
    elif which == "cfg2sso":
        cfg2_sso(sys.argv[2])
    elif which == "cfg4":
        cfg4()
    elif which == "cfg3":  # optional third argument: another output path
        cfg3(int(sys.argv[2]), sys.argv[3] if len(sys.argv) > 3 else None)
    else:
        raise SystemExit(__doc__)
    say("done")
