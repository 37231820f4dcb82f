"""GPU block-Davidson TI-TDA solver (rttda_eigen_lowest, eq. casida_tda) and eigenstate
populations (rttda_populations, eq. populations) against the FP64 oracle's dense eigensolver.

Tolerances: eigenvalues within 1e-5 Ha (FP32 sigma) or 1e-4 Ha (split BF16), the precisions'
bars for spectral peaks; eigenvectors by |overlap| with the oracle's (random spectra are
non-degenerate); populations within 1e-6 (FP32) / 1e-4 (mixed) absolute."""
import numpy as np
import pytest

from conftest import say
from oracle import rttda64 as O
from paper_2601_16949_amd import inputs as I

pytestmark = pytest.mark.gpu

EIG_TOL = {"fp32": 1e-5, "mixed": 1e-4}


def _setup(o, v, nq, prec, seed, max_rhs=2):
    from paper_2601_16949_amd import rttda

    shape = I.Shape(o, v, nq, b_scale=0.05, storage="f32" if prec == "fp32" else "bf16")
    prob = I.make_problem(shape, seed)
    ctx = rttda.Context(rttda.DeviceProblem(prob, prec), max_rhs=max_rhs)
    return O.Operator.from_problem(prob), ctx


@pytest.mark.parametrize("o,v,nq,k,prec,max_rhs", [(10, 40, 120, 6, "fp32", 1), (3, 4, 2, 2, "fp32", 1),
                                                    (24, 96, 64, 8, "mixed", 3), (40, 120, 80, 10, "fp32", 2),
                                                    (17, 67, 0, 5, "fp32", 1), (30, 96, 40, 4, "mixed", 1)])
def test_eigen_lowest_matches_oracle(gpu_lib, o, v, nq, k, prec, max_rhs):
    op, ctx = _setup(o, v, nq, prec, 900 + o, max_rhs)
    tol = 1e-6 if prec == "fp32" else 2e-5
    w, res, U, its = ctx.eigen_lowest(k, tol=tol, max_iter=300)
    say(f"[davidson] o={o} v={v} nq={nq} k={k} {prec}: {its} iterations, max residual {res.max():.2e}")
    wo, Uo = O.lowest_states(op, k)
    assert np.all(res <= tol), res
    assert np.all(np.diff(w) >= -1e-12)
    assert np.max(np.abs(w - wo)) <= EIG_TOL[prec], (w, wo)
    Ug = U.cpu().numpy().reshape(k, -1)
    norms = np.linalg.norm(Ug, axis=1)
    assert np.allclose(norms, 1.0, atol=1e-10)
    gaps = np.diff(np.concatenate([[-np.inf], wo, [np.inf]]))
    for j in range(k):
        if min(gaps[j], gaps[j + 1]) < 1e-3:
            continue  # a near-degenerate pair: only the span is defined
        ov = abs(float(Ug[j] @ Uo[:, j]))
        assert ov >= 1 - (1e-6 if prec == "fp32" else 1e-4), (j, ov)


def test_eigen_lowest_argument_errors(gpu_lib):
    _, ctx = _setup(5, 9, 3, "fp32", 17)
    for bad in (dict(k=0), dict(k=3, m_max=5), dict(k=2, m_max=100), dict(k=2, tol=0.0), dict(k=2, max_iter=0)):
        with pytest.raises(gpu_lib.RttdaError):
            ctx.eigen_lowest(**{"m_max": 0, **bad})


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_populations_match_oracle(gpu_lib, prec):
    """Populations of the 8 lowest states after 40 steps of a kicked propagation: the device
    projection of the GPU state on the GPU eigenvectors against the oracle's projection of the
    oracle state on its eigenvectors."""
    import torch

    o, v, nq = 12, 48, 60
    op, ctx = _setup(o, v, nq, prec, 4321, max_rhs=2)
    k = 8
    w, res, U, _ = ctx.eigen_lowest(k, tol=1e-6 if prec == "fp32" else 2e-5, max_iter=300)
    pulses = I.kick_pulses(axes=[(0.0, 0.0, 1.0), (1.0, 0.0, 0.0)], kappa=1e-2)
    c0d, cd = gpu_lib.ground_state(2, o, v)
    ctx.propagate(pulses, 0.05, 40, c0d, cd, want_trace=False)
    torch.cuda.synchronize()
    got = ctx.populations(U, cd)
    wo, Uo = O.lowest_states(op, k)
    Ug = U.cpu().numpy().reshape(k, -1)
    sign = np.sign(np.sum(Ug * Uo.T, axis=1))
    for r, p in enumerate(pulses):
        blocks = O.dipole_blocks(op, p.direction)
        c0, C = O.kick(blocks, p.e0, 1.0 + 0j, np.zeros((o, v), complex))
        for n in range(40):
            c0, C = O.rk4_step(op, blocks, p, 0.05, n, c0, C)
        ref = O.state_populations(Uo, c0, C)[1:]
        # the Ritz vector's error is at most resid/gap in norm, so |<U, c>| moves by at most
        # (resid/gap) |C|; the state itself carries the propagation's relative error
        gaps = np.array([np.min(np.abs(np.delete(np.linalg.eigvalsh(O.dense_A(op)), j) - wo[j])) for j in range(k)])
        du = res / gaps * np.linalg.norm(C)
        tol = 2 * np.sqrt(ref) * du + du ** 2 + (1e-6 if prec == "fp32" else 1e-4) * np.max(ref)
        err = np.abs(got[r] - ref)
        say(f"[populations] {prec} rhs {r}: max |P_gpu - P_ora| = {err.max():.2e}, worst err/bound "
            f"{np.max(err / tol):.2f} (max P {np.max(ref):.2e})")
        assert np.all(err <= tol)
        assert np.all(sign != 0)
        # tight check of the projection itself: the oracle state on the GPU's eigenvectors
        own = np.abs(Ug @ np.asarray(C).reshape(-1)) ** 2
        e2 = np.abs(got[r] - own)
        say(f"[populations] {prec} rhs {r}: projection on the GPU vectors, max error {e2.max():.2e}")
        assert np.all(e2 <= 1e-12 + (1e-6 if prec == "fp32" else 1e-4) * np.max(own))


@pytest.mark.parametrize("integrator", ["rk4", "sso"])
def test_populations_output_of_propagation(gpu_lib, integrator):
    """Populations as a per-step output of the propagation (rttda_set_populations): every sample
    against the oracle trajectory projected on the same (GPU) eigenvectors, and the last sample
    against the separate projection call."""
    import torch

    o, v, nq, n, k = 12, 48, 60, 60, 6
    op, ctx = _setup(o, v, nq, "fp32", 4321, max_rhs=2)
    _, _, U, _ = ctx.eigen_lowest(k, tol=1e-6, max_iter=300)
    pulses = I.kick_pulses(axes=[(0.0, 0.0, 1.0), (0.0, 1.0, 0.0)], kappa=1e-2)
    c0d, cd = gpu_lib.ground_state(2, o, v)
    pops = torch.full((n + 1, 2, k), float("nan"), dtype=torch.float64, device="cuda")
    ctx.propagate(pulses, 0.05, n, c0d, cd, want_trace=False, integrator=integrator, pops=pops, pop_vectors=U)
    torch.cuda.synchronize()
    got = pops.cpu().numpy()
    assert np.isfinite(got).all()
    last = ctx.populations(U, cd)
    assert np.max(np.abs(got[-1] - last)) <= 1e-14 * np.max(last)
    Ug = U.cpu().numpy().reshape(k, -1)
    for r, p in enumerate(pulses):
        blocks = O.dipole_blocks(op, p.direction)
        c0, C = O.kick(blocks, p.e0, 1.0 + 0j, np.zeros((o, v), complex))
        q0, Q, p0, P = c0.real, C.real.copy(), c0.imag, C.imag.copy()
        worst = 0.0
        for step in range(n + 1):
            ref = np.abs(Ug @ C.reshape(-1)) ** 2
            err = np.max(np.abs(got[step, r] - ref))
            worst = max(worst, err / (1e-12 + 1e-6 * np.max(ref)))
            assert err <= 1e-12 + 1e-6 * np.max(ref), (step, r, err)
            if step < n:
                if integrator == "rk4":
                    c0, C = O.rk4_step(op, blocks, p, 0.05, step, c0, C)
                else:
                    q0, Q, p0, P = O.sso_step(op, blocks, p, 0.05, step, q0, Q, p0, P)
                    c0, C = complex(q0, p0), Q + 1j * P
        say(f"[populations output] {integrator} rhs {r}: worst error / bound {worst:.3f}")
