"""FP64 oracle for the RT-TDA hot path (test infrastructure only).

What it computes, and where the paper defines it (Knoll & Levine, "GPU-accelerated
real-time Tamm-Dancoff approximation", arxiv 2601.16949):

* The TDA matrix A (Theory and Methods, eq. A_matrix_element2), taken in
  density-fitted form with a hybrid exchange term and without the f_xc kernel:
      A_{ia,jb} = delta_ij delta_ab (e_a - e_i) + 2 sum_Q B^Q_ia B^Q_jb
                  - c_x sum_Q B^Q_ij B^Q_ab
  with ia in virtuals-run-fastest order (text after eq. A_matrix_element2).
* The extended space with the Kohn-Sham ground state as element 0 and
  A_{0,ia} = 0 (Real-Time TDA subsection, text after eq. ode_rt_tda).  A_00 is
  read as 0 so that spectral peaks sit at the excitation energies (the
  F-coronene excitation-energy table compares peaks with TI-TDA energies).
* The dipole coupling (eqs. e_field, sigmas): H(t) = A_0 - E(t) mu.d, with mu
  mapped from the MO basis to CSFs by the Slater-Condon rules (eqs. sc1-sc6).
  The constant <Phi0|mu|Phi0> (sc1, sc3) acts as a multiple of the identity on
  the whole space and is dropped.
* The time-dependent Schroedinger equation i dX/dt = H(t) X (eq. ode_rt_tda),
  integrated with the classic 4-stage Runge-Kutta method (the paper uses a
  split-operator integrator; this path uses RK4), with fields evaluated at
  t, t+dt/2, t+dt/2, t+dt where t = n dt.
* Pulses (eqs. delta_pulse, continuous wave, transform_limited, chirped_pulse),
  sigma = FWHM / 2.35482.  The delta pulse is applied as a first-order kick
  X <- X + i kappa mu.d X before the first step (text on the delta pulse in the
  Propagation Algorithm subsection: the response stays linear in the pulse).
* The observable: the dipole trace mu(t_n) = Re <X_n | mu.d | X_n>, and the norm.
* The paper's own integrator, second-order symplectic split operator on X = q + i p
  (Propagation Algorithm subsection), as a second propagation route.

Arrays: a state is (c0, C) with c0 complex scalar and C complex (o, v).
"""
from __future__ import annotations

import math

import numpy as np

SQRT2 = math.sqrt(2.0)
FWHM_TO_SIGMA = 2.35482

PULSE_NONE, PULSE_DELTA, PULSE_CW, PULSE_GAUSS, PULSE_CHIRP, PULSE_DELTA_EXACT = 0, 1, 2, 3, 4, 5


class BF16Stored:
    """Factors kept as their stored BF16 bit patterns (uint16, [N_Q, ...]) and read back as FP64
    one range of Q at a time, for shapes whose FP64 copy would not fit in host memory.  A BF16
    value is the upper half of the FP32 with the same bits, so the read is exact."""

    def __init__(self, bits: np.ndarray):
        if bits.dtype != np.uint16:
            raise TypeError("BF16Stored takes uint16 bit patterns")
        self.bits = bits
        self.shape = bits.shape

    def __getitem__(self, index):
        return (self.bits[index].astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _factor(b):
    return b if isinstance(b, BF16Stored) else np.asarray(b, dtype=np.float64)


class Operator:
    """FP64 copies of the stored inputs of one molecule (factors also as BF16Stored, read per Q
    range)."""

    def __init__(self, e_occ, e_virt, b_ov, b_oo, b_vv, mu, cx):
        self.e_occ = np.asarray(e_occ, dtype=np.float64)
        self.e_virt = np.asarray(e_virt, dtype=np.float64)
        self.b_ov = _factor(b_ov)
        self.b_oo = _factor(b_oo)
        self.b_vv = _factor(b_vv)
        self.mu = np.asarray(mu, dtype=np.float64)
        self.cx = float(cx)
        self.o = self.e_occ.shape[0]
        self.v = self.e_virt.shape[0]
        self.nq = self.b_ov.shape[0]

    @classmethod
    def from_problem(cls, p):
        return cls(p.e_occ, p.e_virt, p.b_ov, p.b_oo, p.b_vv, p.mu, p.cx)


# ----------------------------------------------------------------------------------------
# A applied to a real o x v amplitude matrix (eq. A_matrix_element2, DF form)
# ----------------------------------------------------------------------------------------
def orbital_gaps(op: Operator) -> np.ndarray:
    """D_ia = e_a - e_i: the diagonal term delta_ij delta_ab (e_a - e_i)."""
    return op.e_virt[None, :] - op.e_occ[:, None]


def coulomb(op: Operator, C: np.ndarray, q_chunk: int = 256) -> np.ndarray:
    """J_ia = 2 sum_jb (ia|jb) C_jb with (ia|jb) = sum_Q B^Q_ia B^Q_jb, as
    d_Q = sum_jb B^Q_jb C_jb and J = 2 sum_Q d_Q B^Q, the sum over Q taken a range of Q at a time.
    C may carry leading dimensions (several real planes at once)."""
    J = np.zeros_like(C)
    for q0 in range(0, op.nq, q_chunk):
        B = op.b_ov[q0:min(op.nq, q0 + q_chunk)]
        d = np.einsum("qjb,...jb->...q", B, C)
        J += 2.0 * np.einsum("...q,qia->...ia", d, B)
    return J


def exchange(op: Operator, C: np.ndarray, q_chunk: int = 64) -> np.ndarray:
    """K_ia = sum_jb (ij|ab) C_jb = sum_Q (B^Q_oo C B^Q_vv)_ia, (ij|ab) = sum_Q B^Q_ij B^Q_ab.
    C may carry one leading dimension (several real planes at once)."""
    Cb = C.reshape((-1,) + C.shape[-2:])  # (planes, o, v)
    K = np.zeros_like(Cb)
    for q0 in range(0, op.nq, q_chunk):
        q1 = min(op.nq, q0 + q_chunk)
        V = np.matmul(op.b_oo[q0:q1][:, None], Cb[None])  # (nq_chunk, planes, o, v)
        K += np.matmul(V, op.b_vv[q0:q1][:, None]).sum(axis=0)
    return K.reshape(C.shape)


def apply_A_real(op: Operator, C: np.ndarray) -> np.ndarray:
    return orbital_gaps(op) * C + coulomb(op, C) - op.cx * exchange(op, C)


def apply_A(op: Operator, C: np.ndarray) -> np.ndarray:
    """A is real, so it acts on the real and imaginary parts of C separately (both planes in one
    pass over the factors)."""
    if np.iscomplexobj(C):
        planes = apply_A_real(op, np.stack([C.real, C.imag]))
        return planes[0] + 1j * planes[1]
    return apply_A_real(op, C)


# ----------------------------------------------------------------------------------------
# Dipole coupling (eqs. e_field, sc1-sc6)
# ----------------------------------------------------------------------------------------
def dipole_along(op: Operator, direction) -> np.ndarray:
    d = np.asarray(direction, dtype=np.float64)
    return np.einsum("k,kpq->pq", d, op.mu)


def dipole_blocks(op: Operator, direction):
    m = dipole_along(op, direction)
    o = op.o
    return m[:o, :o], m[:o, o:], m[o:, o:]


def apply_dipole(blocks, c0, C):
    """(M X) for X = (c0, C), M the CSF-basis dipole from the Slater-Condon rules:
    (M X)_0  = sqrt2 sum_ia mu_ia c_ia                              (sc2)
    (M X)_ia = sqrt2 mu_ia c0 + sum_b mu_ab c_ib - sum_j mu_ij c_ja  (sc2, sc3-sc5; sc6 -> 0)
    The i=j, a=b terms of the last two sums give the diagonal mu_aa - mu_ii (sc3)."""
    moo, mov, mvv = blocks
    g = SQRT2 * np.sum(mov * C)
    F = C @ mvv - moo @ C + SQRT2 * mov * c0
    return g, F


def dense_dipole_csf(op: Operator, direction) -> np.ndarray:
    """Dense (1+ov) x (1+ov) CSF-basis dipole written rule by rule (eqs. sc1-sc6),
    with <Phi0|mu|Phi0> dropped.  Pure Python loops: tiny inputs only."""
    moo, mov, mvv = dipole_blocks(op, direction)
    o, v = op.o, op.v
    n = o * v
    M = np.zeros((n + 1, n + 1))
    for i in range(o):
        for a in range(v):
            ia = 1 + i * v + a
            M[0, ia] = M[ia, 0] = SQRT2 * mov[i, a]  # sc2
            for j in range(o):
                for b in range(v):
                    jb = 1 + j * v + b
                    if i == j and a == b:
                        M[ia, jb] = mvv[a, a] - moo[i, i]  # sc3 minus <Phi0|mu|Phi0>
                    elif i == j:
                        M[ia, jb] = mvv[a, b]  # sc4
                    elif a == b:
                        M[ia, jb] = -moo[i, j]  # sc5
                    # else sc6: 0
    return M


def dense_dipole_csf_fast(op: Operator, direction) -> np.ndarray:
    """Same matrix as dense_dipole_csf, assembled with Kronecker products (for larger ov)."""
    moo, mov, mvv = dipole_blocks(op, direction)
    o, v = op.o, op.v
    n = o * v
    M = np.zeros((n + 1, n + 1))
    M[0, 1:] = SQRT2 * mov.reshape(-1)
    M[1:, 0] = M[0, 1:]
    M[1:, 1:] = np.kron(np.eye(o), mvv) - np.kron(moo, np.eye(v))
    return M


# ----------------------------------------------------------------------------------------
# Dense A (explicit four-index integrals) -- the definition written out
# ----------------------------------------------------------------------------------------
def eri_ovov(op: Operator) -> np.ndarray:
    """(ia|jb) = sum_Q B^Q_ia B^Q_jb as a 4-index array [i,a,j,b]."""
    return np.einsum("qia,qjb->iajb", op.b_ov, op.b_ov)


def eri_oovv(op: Operator) -> np.ndarray:
    """(ij|ab) = sum_Q B^Q_ij B^Q_ab as a 4-index array [i,j,a,b]."""
    return np.einsum("qij,qab->ijab", op.b_oo, op.b_vv)


def dense_A(op: Operator) -> np.ndarray:
    o, v = op.o, op.v
    A = 2.0 * eri_ovov(op) - op.cx * eri_oovv(op).transpose(0, 2, 1, 3)
    A = A.reshape(o * v, o * v)
    A[np.diag_indices(o * v)] += orbital_gaps(op).reshape(-1)
    return A


def dense_A_blas(op: Operator) -> np.ndarray:
    """dense_A assembled through two GEMMs (for ov in the tens of thousands)."""
    o, v, nq = op.o, op.v, op.nq
    Bov = op.b_ov.reshape(nq, o * v)
    A = 2.0 * (Bov.T @ Bov)
    X = (op.b_oo.reshape(nq, o * o).T @ op.b_vv.reshape(nq, v * v))  # [(i,j),(a,b)]
    A -= op.cx * X.reshape(o, o, v, v).transpose(0, 2, 1, 3).reshape(o * v, o * v)
    A[np.diag_indices(o * v)] += orbital_gaps(op).reshape(-1)
    return A


# ----------------------------------------------------------------------------------------
# Pulses (eqs. delta_pulse .. chirped_pulse)
# ----------------------------------------------------------------------------------------
def field_value(p, t: float) -> float:
    """E(t) of a continuous pulse; 0 for the delta pulse (it acts as a kick at t = 0)."""
    kind = p.kind
    if kind in (PULSE_NONE, PULSE_DELTA, PULSE_DELTA_EXACT):
        return 0.0
    if kind == PULSE_CW:
        return p.e0 * math.sin(p.omega * t + p.phase)
    s = p.fwhm / FWHM_TO_SIGMA
    tau = t - p.t0
    env = math.exp(-tau * tau / (2.0 * s * s))
    if kind == PULSE_GAUSS:
        return p.e0 * env * math.sin(p.omega * tau + p.phase)
    if kind == PULSE_CHIRP:
        return p.e0 * env * math.sin((p.omega + 0.5 * p.beta * tau) * tau + p.phase)
    raise ValueError(f"unknown pulse kind {kind}")


# ----------------------------------------------------------------------------------------
# H(t) X, kick, observables
# ----------------------------------------------------------------------------------------
def apply_H(op: Operator, blocks, E: float, c0, C):
    """H X with H = diag(0, A) - E M (eq. e_field): returns ((H X)_0, (H X)_C)."""
    g, F = apply_dipole(blocks, c0, C)
    return -E * g, apply_A(op, C) - E * F


def kick(blocks, kappa: float, c0, C):
    """First-order delta kick X <- X + i kappa M X."""
    g, F = apply_dipole(blocks, c0, C)
    return c0 + 1j * kappa * g, C + 1j * kappa * F


def kick_exact(op: "Operator", direction, kappa: float, c0, C):
    """Unitary delta kick X <- exp(i kappa M) X: the exact propagator of a delta field of area
    kappa, from the dense CSF dipole and the matrix exponential (small inputs)."""
    import scipy.linalg

    M = dense_dipole_csf_fast(op, direction)
    x = np.concatenate([[complex(c0)], np.asarray(C, dtype=np.complex128).reshape(-1)])
    y = scipy.linalg.expm(1j * kappa * M) @ x
    return y[0], y[1:].reshape(op.o, op.v)


def apply_kick(op: "Operator", blocks, pulse, c0, C):
    """The kick of a delta pulse (first order or exact); other pulses leave the state alone."""
    if pulse.kind == PULSE_DELTA:
        return kick(blocks, pulse.e0, c0, C)
    if pulse.kind == PULSE_DELTA_EXACT:
        return kick_exact(op, pulse.direction, pulse.e0, c0, C)
    return c0, C


def dipole_expectation(blocks, c0, C) -> float:
    """Re <X | M | X>."""
    g, F = apply_dipole(blocks, c0, C)
    return float((np.conj(c0) * g).real + np.sum(np.conj(C) * F).real)


def norm2(c0, C) -> float:
    return float(abs(c0) ** 2 + np.sum(np.abs(C) ** 2))


def energy(op: Operator, c0, C) -> float:
    """<X | diag(0, A) | X>."""
    return float(np.sum(np.conj(C) * apply_A(op, C)).real)


# ----------------------------------------------------------------------------------------
# RK4 propagation, direct route (O1)
# ----------------------------------------------------------------------------------------
RK4_NODES = (0.0, 0.5, 0.5, 1.0)


def rk4_step(op: Operator, blocks, pulse, dt: float, n: int, c0, C):
    """One classic RK4 step of dX/dt = -i H(t) X from t = n dt."""

    def f(frac, y0, Y):
        t = (n + frac) * dt
        h0, hC = apply_H(op, blocks, field_value(pulse, t), y0, Y)
        return -1j * h0, -1j * hC

    k1 = f(0.0, c0, C)
    k2 = f(0.5, c0 + 0.5 * dt * k1[0], C + 0.5 * dt * k1[1])
    k3 = f(0.5, c0 + 0.5 * dt * k2[0], C + 0.5 * dt * k2[1])
    k4 = f(1.0, c0 + dt * k3[0], C + dt * k3[1])
    c0n = c0 + dt / 6.0 * (k1[0] + 2.0 * k2[0] + 2.0 * k3[0] + k4[0])
    Cn = C + dt / 6.0 * (k1[1] + 2.0 * k2[1] + 2.0 * k3[1] + k4[1])
    return c0n, Cn


def propagate(op: Operator, pulse, dt: float, n_steps: int, c0=1.0 + 0j, C=None, step0: int = 0,
              want_norm: bool = False):
    """Propagate one right-hand side; returns (trace[n_steps+1], c0, C[, norms]).

    Starts from the Kohn-Sham ground state (c0 = 1, C = 0) unless given.  A delta
    pulse kicks the state once when step0 == 0."""
    if C is None:
        C = np.zeros((op.o, op.v), dtype=np.complex128)
    c0 = complex(c0)
    C = np.array(C, dtype=np.complex128)
    blocks = dipole_blocks(op, pulse.direction)
    if step0 == 0:
        c0, C = apply_kick(op, blocks, pulse, c0, C)
    trace = np.empty(n_steps + 1)
    norms = np.empty(n_steps + 1)
    trace[0] = dipole_expectation(blocks, c0, C)
    norms[0] = norm2(c0, C)
    for n in range(n_steps):
        c0, C = rk4_step(op, blocks, pulse, dt, step0 + n, c0, C)
        trace[n + 1] = dipole_expectation(blocks, c0, C)
        norms[n + 1] = norm2(c0, C)
    if want_norm:
        return trace, c0, C, norms
    return trace, c0, C


# ----------------------------------------------------------------------------------------
# Second-order symplectic split-operator (SSO) propagation (Propagation Algorithm
# subsection: X = q + i p, eq. x_real_imagiary; dq/dt = H p, dp/dt = -H q)
# ----------------------------------------------------------------------------------------
def apply_H_real(op: Operator, blocks, E: float, x0: float, X: np.ndarray):
    """H(t) x for a real vector x = (x0, X); H is real symmetric, so the result is real."""
    h0, hX = apply_H(op, blocks, E, x0, X)
    return float(np.real(h0)), np.real(hX)


def sso_step(op: Operator, blocks, pulse, dt: float, n: int, q0, Q, p0, P):
    """One symmetric kick-drift-kick step from t = n dt of the symplectic form:
        p <- p - dt/2 H(t_n) q;   q <- q + dt H(t_n + dt/2) p;   p <- p - dt/2 H(t_n + dt) q."""
    h0, hQ = apply_H_real(op, blocks, field_value(pulse, n * dt), q0, Q)
    p0, P = p0 - 0.5 * dt * h0, P - 0.5 * dt * hQ
    g0, gP = apply_H_real(op, blocks, field_value(pulse, (n + 0.5) * dt), p0, P)
    q0, Q = q0 + dt * g0, Q + dt * gP
    h0, hQ = apply_H_real(op, blocks, field_value(pulse, (n + 1) * dt), q0, Q)
    p0, P = p0 - 0.5 * dt * h0, P - 0.5 * dt * hQ
    return q0, Q, p0, P


def propagate_sso(op: Operator, pulse, dt: float, n_steps: int, c0=1.0 + 0j, C=None, step0: int = 0,
                  want_norm: bool = False):
    """As propagate() with the SSO step instead of RK4 (same kick, trace and norm)."""
    if C is None:
        C = np.zeros((op.o, op.v), dtype=np.complex128)
    c0 = complex(c0)
    C = np.array(C, dtype=np.complex128)
    blocks = dipole_blocks(op, pulse.direction)
    if step0 == 0:
        c0, C = apply_kick(op, blocks, pulse, c0, C)
    q0, Q, p0, P = c0.real, C.real.copy(), c0.imag, C.imag.copy()
    trace = np.empty(n_steps + 1)
    norms = np.empty(n_steps + 1)
    trace[0] = dipole_expectation(blocks, c0, C)
    norms[0] = norm2(c0, C)
    for n in range(n_steps):
        q0, Q, p0, P = sso_step(op, blocks, pulse, dt, step0 + n, q0, Q, p0, P)
        c0, C = complex(q0, p0), Q + 1j * P
        trace[n + 1] = dipole_expectation(blocks, c0, C)
        norms[n + 1] = norm2(c0, C)
    if want_norm:
        return trace, c0, C, norms
    return trace, c0, C


def correlation(c0ref, Cref, c0, C) -> complex:
    """Time-correlation function (eq. time_correlation_function): <X_ref | X>, the sum over the
    ground amplitude and the amplitudes c_ia of conj(reference) times state."""
    return complex(np.conj(complex(c0ref)) * complex(c0)
                   + np.vdot(np.asarray(Cref, dtype=np.complex128).reshape(-1),
                             np.asarray(C, dtype=np.complex128).reshape(-1)))


def propagate_correlation(op: Operator, pulse, dt: float, n_steps: int, integrator: str = "rk4"):
    """R(t_n) = <X(0+) | X(t_n)> for n = 0..n_steps from the ground state, X(0+) being the state
    after the delta kick (direct route, RK4 or the split operator)."""
    blocks = dipole_blocks(op, pulse.direction)
    c0, C = apply_kick(op, blocks, pulse, 1.0 + 0j, np.zeros((op.o, op.v), dtype=np.complex128))
    r0, R0 = c0, C.copy()
    out = np.empty(n_steps + 1, dtype=np.complex128)
    out[0] = correlation(r0, R0, c0, C)
    q0, Q, p0, P = c0.real, C.real.copy(), c0.imag, C.imag.copy()
    for n in range(n_steps):
        if integrator == "rk4":
            c0, C = rk4_step(op, blocks, pulse, dt, n, c0, C)
        else:
            q0, Q, p0, P = sso_step(op, blocks, pulse, dt, n, q0, Q, p0, P)
            c0, C = complex(q0, p0), Q + 1j * P
        out[n + 1] = correlation(r0, R0, c0, C)
    return out


def sso_mode_matrix(a: float) -> np.ndarray:
    """The SSO step acting on one field-free eigenmode (q, p) of frequency w, a = w dt."""
    return np.array([[1.0 - a * a / 2.0, a], [-a * (1.0 - a * a / 4.0), 1.0 - a * a / 2.0]])


# ----------------------------------------------------------------------------------------
# Eigen route (O2): dense A, eigh, and RK4 in the eigenbasis
# ----------------------------------------------------------------------------------------
def rk4_amplification(z):
    """Stability polynomial of classic RK4: R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24."""
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def lowest_states(op: Operator, k: int):
    """The k lowest TI-TDA states (eigenpairs of A, eq. casida_tda): energies w[k] and
    eigenvectors U[(i,a), k], from the dense A and a LAPACK subset eigensolver."""
    import scipy.linalg

    A = dense_A_blas(op) if op.o * op.v > 600 else dense_A(op)
    w, U = scipy.linalg.eigh(A, subset_by_index=[0, k - 1])
    return w, U


def state_populations(U: np.ndarray, c0, C) -> np.ndarray:
    """Populations of the ground state and of the TI-TDA states in the columns of U by projection
    of the amplitudes (eq. populations): [|c0|^2, |U_1^T c|^2, ...]."""
    x = np.asarray(C, dtype=np.complex128).reshape(-1)
    return np.concatenate([[abs(complex(c0)) ** 2], np.abs(U.T @ x) ** 2])


class EigenRoute:
    """Extended-space eigen decomposition: w[0] = 0 (ground state), w[1:] = eig(A)."""

    def __init__(self, op: Operator, A=None):
        if A is None:
            A = dense_A_blas(op) if op.o * op.v > 600 else dense_A(op)
        w, U = np.linalg.eigh(A)
        n = op.o * op.v
        self.op = op
        self.w = np.concatenate([[0.0], w])
        self.U = np.zeros((n + 1, n + 1))
        self.U[0, 0] = 1.0
        self.U[1:, 1:] = U

    def to_eig(self, c0, C):
        x = np.concatenate([[complex(c0)], np.asarray(C, dtype=np.complex128).reshape(-1)])
        return self.U.T @ x

    def from_eig(self, y):
        x = self.U @ y
        return x[0], x[1:].reshape(self.op.o, self.op.v)

    def dipole_eig(self, direction):
        M = dense_dipole_csf_fast(self.op, direction)
        return self.U.T @ M @ self.U

    def propagate_field_free(self, pulse, dt: float, n_steps: int, c0=1.0 + 0j, C=None,
                             want_state: bool = False):
        """Exact RK4 map for field-free steps: y_n = R(-i w dt)^n y_0 (after the kick)."""
        if C is None:
            C = np.zeros((self.op.o, self.op.v), dtype=np.complex128)
        blocks = dipole_blocks(self.op, pulse.direction)
        if pulse.kind in (PULSE_DELTA, PULSE_DELTA_EXACT):
            c0, C = apply_kick(self.op, blocks, pulse, complex(c0), np.asarray(C, dtype=np.complex128))
        elif pulse.kind != PULSE_NONE:
            raise ValueError("field-free route takes only delta or no pulse")
        y = self.to_eig(c0, C)
        Me = self.dipole_eig(pulse.direction)
        R = rk4_amplification(-1j * self.w * dt)
        trace = np.empty(n_steps + 1)
        # trace[n] = Re y_n^H Me y_n with y_{n+1} = R y_n, evaluated for a block of steps at a
        # time (one matrix product per block instead of one matrix-vector product per step)
        block = 256
        for n0 in range(0, n_steps + 1, block):
            nb = min(block, n_steps + 1 - n0)
            Y = np.empty((nb, y.size), dtype=np.complex128)
            for k in range(nb):
                Y[k] = y
                if n0 + k < n_steps:
                    y = R * y
            trace[n0:n0 + nb] = np.real(np.sum(np.conj(Y) * (Y @ Me), axis=1))
        if want_state:
            return trace, y
        return trace

    def field_free_trace_blocked(self, pulse, dt: float, n_steps: int, c0=1.0 + 0j, C=None, block: int = 256):
        """The same trace as propagate_field_free, trace[n] = Re <X_n | M | X_n> with the exact
        field-free RK4 map y_n = R(-i w dt)^n y_0, evaluated for large ov: each block of steps is
        taken back to the amplitude basis, X_n = U y_n (one matrix product per block), and M acts
        there in its factorised form (apply_dipole), so the dense eigenbasis dipole U^T M U is
        never formed."""
        if C is None:
            C = np.zeros((self.op.o, self.op.v), dtype=np.complex128)
        blocks = dipole_blocks(self.op, pulse.direction)
        if pulse.kind in (PULSE_DELTA, PULSE_DELTA_EXACT):
            c0, C = apply_kick(self.op, blocks, pulse, complex(c0), np.asarray(C, dtype=np.complex128))
        elif pulse.kind != PULSE_NONE:
            raise ValueError("field-free route takes only delta or no pulse")
        y = self.to_eig(c0, C)
        R = rk4_amplification(-1j * self.w * dt)
        logR = np.log(R)
        Uexc = np.ascontiguousarray(self.U[1:, 1:])  # (BLAS takes contiguous operands only)
        o, v = self.op.o, self.op.v
        moo, mov, mvv = blocks
        trace = np.empty(n_steps + 1)
        for n0 in range(0, n_steps + 1, block):
            n = np.arange(n0, min(n_steps + 1, n0 + block))
            Y = np.exp(np.outer(n, logR)) * y[None, :]  # rows: y_n = R^n y_0
            Yr, Yi = np.ascontiguousarray(Y[:, 1:].real), np.ascontiguousarray(Y[:, 1:].imag)
            Xc = (Yr @ Uexc.T) + 1j * (Yi @ Uexc.T)  # amplitudes C_n (rows)
            # Re <X_n | M | X_n> for the whole block, M X by the same rules as apply_dipole
            C = Xc.reshape(n.size, o, v)
            c0 = Y[:, 0]
            F = (Xc.reshape(n.size * o, v) @ mvv).reshape(n.size, o, v) - np.matmul(moo, C) \
                + SQRT2 * mov[None] * c0[:, None, None]
            g = SQRT2 * np.sum(mov[None] * C, axis=(1, 2))
            trace[n] = (np.conj(c0) * g).real + np.sum(np.conj(C) * F, axis=(1, 2)).real
        return trace

    def field_free_trace_sso_blocked(self, pulse, dt: float, n_steps: int, c0=1.0 + 0j, C=None, block: int = 256):
        """The dipole trace of the split-operator route (propagate_sso) for field-free steps after
        a kick, through the eigenbasis: H = diag(0, A) is real, so q = Re X and p = Im X go to the
        eigenbasis separately and each mode (q_I, p_I) of frequency w_I follows the SSO mode map
        M = sso_mode_matrix(w_I dt), whose determinant is 1.  With cos(th) = 1 - a^2/2 (a < 2) the
        powers are M^n = s_n M - s_(n-1) 1, s_n = sin(n th) / sin(th) (the two-term recurrence of a
        unimodular 2 x 2 matrix); the ground mode (w = 0) has M = 1.  Each block of steps returns to
        the amplitude basis and M acts there in factorised form, as in field_free_trace_blocked."""
        if C is None:
            C = np.zeros((self.op.o, self.op.v), dtype=np.complex128)
        blocks = dipole_blocks(self.op, pulse.direction)
        if pulse.kind in (PULSE_DELTA, PULSE_DELTA_EXACT):
            c0, C = apply_kick(self.op, blocks, pulse, complex(c0), np.asarray(C, dtype=np.complex128))
        elif pulse.kind != PULSE_NONE:
            raise ValueError("field-free route takes only delta or no pulse")
        y = self.to_eig(c0, C)
        qy, py = y.real, y.imag  # U is real: the real and imaginary parts transform separately
        a = self.w * dt
        if np.any(a[1:] >= 2.0):
            raise ValueError("split operator unstable: w dt >= 2")
        m11 = 1.0 - a * a / 2.0
        m12 = a
        m21 = -a * (1.0 - a * a / 4.0)
        th = np.arccos(np.clip(m11, -1.0, 1.0))
        live = th > 0.0
        sin_th = np.where(live, np.sin(th), 1.0)
        Uexc = np.ascontiguousarray(self.U[1:, 1:])
        o, v = self.op.o, self.op.v
        moo, mov, mvv = blocks
        trace = np.empty(n_steps + 1)
        for n0 in range(0, n_steps + 1, block):
            n = np.arange(n0, min(n_steps + 1, n0 + block))
            s_n = np.where(live[None, :], np.sin(np.outer(n, th)) / sin_th[None, :], n[:, None].astype(float))
            s_m = np.where(live[None, :], np.sin(np.outer(n - 1, th)) / sin_th[None, :], (n[:, None] - 1.0))
            # M^n = s_n M - s_(n-1) 1 (for w = 0: M = 1 and s_n = n, so M^n = n 1 - (n - 1) 1 = 1)
            Qy = (s_n * m11 - s_m) * qy + (s_n * m12) * py
            Py = (s_n * m21) * qy + (s_n * m11 - s_m) * py
            Xq = np.ascontiguousarray(Qy[:, 1:]) @ Uexc.T
            Xp = np.ascontiguousarray(Py[:, 1:]) @ Uexc.T
            Cn = (Xq + 1j * Xp).reshape(n.size, o, v)
            c0n = Qy[:, 0] + 1j * Py[:, 0]
            F = ((Xq + 1j * Xp).reshape(n.size * o, v) @ mvv).reshape(n.size, o, v) - np.matmul(moo, Cn) \
                + SQRT2 * mov[None] * c0n[:, None, None]
            g = SQRT2 * np.sum(mov[None] * Cn, axis=(1, 2))
            trace[n] = (np.conj(c0n) * g).real + np.sum(np.conj(Cn) * F, axis=(1, 2)).real
        return trace

    def propagate_rk4_many(self, pulses, dt: float, n_steps: int, n_pop: int = 0, pop_every: int = 1,
                           progress=None):
        """RK4 with fields for several right-hand sides that share one polarisation, run in the
        eigenbasis from the ground state (after any delta kick), all RHS as the columns of one
        matrix.  Returns (trace [n_steps+1, R], pops) where pops [n_samples, R, 1 + n_pop] holds
        |y_0|^2 and the populations |y_I|^2 of the n_pop lowest TI-TDA states (eq. populations) at
        steps 0, pop_every, 2 pop_every, ..."""
        d = np.asarray(pulses[0].direction, dtype=np.float64)
        for p in pulses:
            if not np.array_equal(np.asarray(p.direction, dtype=np.float64), d):
                raise ValueError("propagate_rk4_many takes pulses of one polarisation")
        blocks = dipole_blocks(self.op, d)
        Rn = len(pulses)
        Y = np.empty((self.w.size, Rn), dtype=np.complex128)
        for r, p in enumerate(pulses):
            c0, C = apply_kick(self.op, blocks, p, 1.0 + 0j, np.zeros((self.op.o, self.op.v), dtype=np.complex128))
            Y[:, r] = self.to_eig(c0, C)
        Me = self.dipole_eig(d)
        w = self.w[:, None]

        def fields(t):
            return np.array([field_value(p, t) for p in pulses])

        def mul(Y):  # Me Y with the real and imaginary parts as the columns of one real product
            Z = Me @ np.concatenate([Y.real, Y.imag], axis=1)
            return Z[:, :Rn] + 1j * Z[:, Rn:]

        def f(t, Y, MY=None):
            if MY is None:
                MY = mul(Y)
            return -1j * (w * Y - fields(t)[None, :] * MY)

        n_samp = n_steps // pop_every + 1
        trace = np.empty((n_steps + 1, Rn))
        pops = np.empty((n_samp, Rn, 1 + n_pop))
        MY = mul(Y)
        for n in range(n_steps + 1):
            trace[n] = np.real(np.sum(np.conj(Y) * MY, axis=0))
            if n % pop_every == 0:
                pops[n // pop_every] = (np.abs(Y[:1 + n_pop]) ** 2).T
            if n == n_steps:
                break
            k1 = f(n * dt, Y, MY)
            k2 = f((n + 0.5) * dt, Y + 0.5 * dt * k1)
            k3 = f((n + 0.5) * dt, Y + 0.5 * dt * k2)
            k4 = f((n + 1.0) * dt, Y + dt * k3)
            Y = Y + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
            MY = mul(Y)
            if progress is not None and (n + 1) % 1000 == 0:
                progress(n + 1)
        return trace, pops

    def propagate_rk4(self, pulse, dt: float, n_steps: int, c0=1.0 + 0j, C=None):
        """RK4 with a field, run in the eigenbasis (RK4 commutes with the change of basis)."""
        if C is None:
            C = np.zeros((self.op.o, self.op.v), dtype=np.complex128)
        blocks = dipole_blocks(self.op, pulse.direction)
        c0, C = complex(c0), np.asarray(C, dtype=np.complex128)
        c0, C = apply_kick(self.op, blocks, pulse, c0, C)
        y = self.to_eig(c0, C)
        Me = self.dipole_eig(pulse.direction)
        w = self.w

        def f(t, y):
            return -1j * (w * y - field_value(pulse, t) * (Me @ y))

        trace = np.empty(n_steps + 1)
        trace[0] = float(np.real(np.conj(y) @ (Me @ y)))
        for n in range(n_steps):
            k1 = f(n * dt, y)
            k2 = f((n + 0.5) * dt, y + 0.5 * dt * k1)
            k3 = f((n + 0.5) * dt, y + 0.5 * dt * k2)
            k4 = f((n + 1.0) * dt, y + dt * k3)
            y = y + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
            trace[n + 1] = float(np.real(np.conj(y) @ (Me @ y)))
        return trace, y


def linear_kick_trace(w, z, kappa: float, dt: float, n_steps: int, chunk: int = 512) -> np.ndarray:
    """The part of the field-free dipole trace after a first-order kick of strength kappa from the
    ground state that is linear in kappa: with eigenvalues w_J of A and z_J = <U_J, sqrt2 mu_ov.d>
    (the ground-excited dipole elements of the eigenstates), the kicked state in the eigenbasis is
    y_0 = e_0 + i kappa z, the RK4 map multiplies y_J by R(-i w_J dt) per step, and
        mu(t_n) = -2 kappa sum_J z_J^2 Im R(-i w_J dt)^n + O(kappa^2).
    The O(kappa^2) remainder is the excited-excited dipole of the response (not included)."""
    w = np.asarray(w, dtype=np.float64)
    wts = np.asarray(z, dtype=np.float64) ** 2
    logR = np.log(rk4_amplification(-1j * w * dt))
    out = np.empty(n_steps + 1)
    for n0 in range(0, n_steps + 1, chunk):
        n = np.arange(n0, min(n_steps + 1, n0 + chunk))
        out[n] = -2.0 * kappa * (np.exp(np.outer(n, logR)).imag @ wts)
    return out


# ----------------------------------------------------------------------------------------
# Sampled single elements (for full-size checks where whole arrays are too costly)
# ----------------------------------------------------------------------------------------
def sigma_element(op: Operator, C_real: np.ndarray, i: int, a: int, d: np.ndarray = None) -> float:
    """(A C)_ia for one (i, a) of a real C, by direct sums over Q, j, b."""
    if d is None:
        d = coulomb_contraction(op.b_ov, C_real)
    return sigma_element_from_slices(op.e_occ[i], op.e_virt[a], C_real, i, a, op.b_ov[:, i, a], d,
                                     op.b_oo[:, i, :], op.b_vv[:, :, a], op.cx)


def coulomb_contraction(b_ov: np.ndarray, C_real: np.ndarray) -> np.ndarray:
    """d_Q = sum_jb B^Q_jb C_jb."""
    return np.einsum("qjb,jb->q", np.asarray(b_ov, dtype=np.float64), C_real)


def sigma_element_from_slices(e_i, e_a, C_real, i, a, b_ov_ia, d, b_oo_i, b_vv_a, cx) -> float:
    """(A C)_ia from the slices of the factors it needs: B^Q_ia (N_Q,), d_Q (N_Q,),
    B^Q_i. (N_Q, o) and B^Q_.a (N_Q, v).  K_ia = sum_Q sum_b (sum_j B_oo[Q,i,j] C[j,b]) B_vv[Q,b,a]."""
    b_oo_i = np.asarray(b_oo_i, dtype=np.float64)
    b_vv_a = np.asarray(b_vv_a, dtype=np.float64)
    diag = (e_a - e_i) * C_real[i, a]
    J = 2.0 * float(np.dot(np.asarray(b_ov_ia, dtype=np.float64), d))
    t = b_oo_i @ C_real  # (N_Q, v)
    K = float(np.sum(t * b_vv_a))
    return diag + J - cx * K
