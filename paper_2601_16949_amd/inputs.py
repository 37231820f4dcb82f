"""Seeded synthetic inputs for RT-TDA propagation problems.

This module is shared by the FP64 CPU oracle and the HIP path: it only draws
random numbers and rounds them to the storage dtype. It holds none of the
method's arithmetic (no sigma vector, no field term, no integrator).

Recipe (stand-ins for the paper's molecules, whose geometries and integrals are
not available):

* orbital energies: e_i ~ U[-1.0, -0.3] Ha (occupied), e_a ~ U[0.05, 1.5] Ha
  (virtual), each sorted ascending, kept in FP64;
* density-fitting factors B^Q_ov (o x v), B^Q_oo (o x o, symmetric),
  B^Q_vv (v x v, symmetric): N(0,1) * s_eff drawn in FP32, one independent
  stream per (seed, tensor, Q) so any single Q slice can be regenerated alone;
  the symmetric factors keep the upper triangle (with the diagonal) of a full
  square draw and mirror it;
* s_eff = min(s, 1.547 / (sqrt(o v) + sqrt(N_Q))): the literal scale makes the
  Coulomb block's top eigenvalue (Marchenko-Pastur edge 2 s^2 (sqrt(ov) +
  sqrt(N_Q))^2) so large that RK4 at the requested dt diverges; the cap holds
  that edge at 4.79 Ha, which is the value of the smallest configuration;
* dipole matrices: three symmetric (o+v) x (o+v) matrices N(0,1) * 0.5 in FP64,
  one per Cartesian direction (x, y, z);
* storage rounding: FP32 (round to nearest) or BF16 (round to nearest even of
  the FP32 value); the oracle reads exactly the rounded values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 16949
TENSOR_E_OCC, TENSOR_E_VIRT, TENSOR_B_OV, TENSOR_B_OO, TENSOR_B_VV, TENSOR_MU, TENSOR_PULSE = range(7)

# Pulse kinds (the four pulses of the paper's pulse equations, plus none).
PULSE_NONE, PULSE_DELTA, PULSE_CW, PULSE_GAUSS, PULSE_CHIRP, PULSE_DELTA_EXACT = 0, 1, 2, 3, 4, 5


@dataclass
class Pulse:
    """One right-hand side's external field.

    kind:  PULSE_* code.  For PULSE_DELTA (first-order kick) and PULSE_DELTA_EXACT (unitary
           kick exp(i kappa M)), e0 is the kick strength kappa.
    e0:    peak field (au).  omega: carrier (Ha).  t0: envelope centre (au).
    fwhm:  envelope full width at half maximum (au), sigma = fwhm / 2.35482.
    beta:  chirp rate (Ha/au).  phase: carrier phase (rad; pi/2 turns sin into cos).
    direction: polarisation unit vector (3,).
    """

    kind: int = PULSE_NONE
    e0: float = 0.0
    omega: float = 0.0
    t0: float = 0.0
    fwhm: float = 1.0
    beta: float = 0.0
    phase: float = 0.0
    direction: tuple = (0.0, 0.0, 1.0)


@dataclass
class Shape:
    o: int
    v: int
    nq: int
    b_scale: float = 0.05
    mu_scale: float = 0.5
    cx: float = 0.2
    storage: str = "f32"  # "f32" | "bf16"
    rescale: bool = True

    @property
    def s_eff(self) -> float:
        if not self.rescale:
            return self.b_scale
        cap = 1.547 / (math.sqrt(self.o * self.v) + math.sqrt(max(self.nq, 0)))
        return min(self.b_scale, cap)


@dataclass
class Problem:
    """Stored (rounded) inputs. Float arrays hold exactly the stored values."""

    shape: Shape
    seed: int
    e_occ: np.ndarray  # f64 (o,)
    e_virt: np.ndarray  # f64 (v,)
    b_ov: np.ndarray  # f32 (nq, o, v), values exactly representable in `storage`
    b_oo: np.ndarray  # f32 (nq, o, o)
    b_vv: np.ndarray  # f32 (nq, v, v)
    mu: np.ndarray  # f64 (3, o+v, o+v)

    @property
    def o(self):
        return self.shape.o

    @property
    def v(self):
        return self.shape.v

    @property
    def nq(self):
        return self.shape.nq

    @property
    def cx(self):
        return self.shape.cx


def _rng(seed: int, tensor: int, q: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(tensor), int(q)]))


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest BF16 (ties to even); returns FP32.  (For finite values the
    bit pattern plus 0x7FFF plus the kept lowest bit stays below 2^32, so 32-bit arithmetic is exact.)"""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32)
    r = (u + (np.uint32(0x7FFF) + ((u >> 16) & np.uint32(1)))) & np.uint32(0xFFFF0000)
    out = r.view(np.float32)
    # NaN/Inf are not produced by this generator; keep them untouched anyway
    bad = ~np.isfinite(x)
    if bad.any():
        out = out.copy()
        out[bad] = x[bad]
    return out


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Upper 16 bits of FP32 values that are exactly BF16-representable."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    return (x.view(np.uint32) >> 16).astype(np.uint16)


def _store(x: np.ndarray, storage: str) -> np.ndarray:
    if storage == "f32":
        return x.astype(np.float32, copy=False)
    if storage == "bf16":
        return round_bf16(x)
    raise ValueError(f"unknown storage dtype {storage!r}")


_UPPER = {}


def _sym(m: np.ndarray) -> np.ndarray:
    """The upper triangle (with the diagonal) of m mirrored into the lower one."""
    n = m.shape[0]
    mask = _UPPER.get(n)
    if mask is None:
        mask = _UPPER[n] = np.triu(np.ones((n, n), dtype=bool))
    return np.where(mask, m, m.T)


def gen_b_ov(shape: Shape, seed: int, q: int) -> np.ndarray:
    s = np.float32(shape.s_eff)
    x = _rng(seed, TENSOR_B_OV, q).standard_normal((shape.o, shape.v), dtype=np.float32) * s
    return _store(x, shape.storage)


def gen_b_oo(shape: Shape, seed: int, q: int) -> np.ndarray:
    s = np.float32(shape.s_eff)
    x = _sym(_rng(seed, TENSOR_B_OO, q).standard_normal((shape.o, shape.o), dtype=np.float32)) * s
    return _store(x, shape.storage)


def gen_b_vv(shape: Shape, seed: int, q: int) -> np.ndarray:
    s = np.float32(shape.s_eff)
    x = _sym(_rng(seed, TENSOR_B_VV, q).standard_normal((shape.v, shape.v), dtype=np.float32)) * s
    return _store(x, shape.storage)


def gen_mu(shape: Shape, seed: int) -> np.ndarray:
    n = shape.o + shape.v
    out = np.empty((3, n, n), dtype=np.float64)
    for k in range(3):
        out[k] = _sym(_rng(seed, TENSOR_MU, k).standard_normal((n, n))) * shape.mu_scale
    return out


def gen_energies(shape: Shape, seed: int):
    e_occ = np.sort(_rng(seed, TENSOR_E_OCC).uniform(-1.0, -0.3, size=shape.o))
    e_virt = np.sort(_rng(seed, TENSOR_E_VIRT).uniform(0.05, 1.5, size=shape.v))
    return e_occ.astype(np.float64), e_virt.astype(np.float64)


def make_problem(shape: Shape, seed: int) -> Problem:
    e_occ, e_virt = gen_energies(shape, seed)
    o, v, nq = shape.o, shape.v, shape.nq
    b_ov = np.empty((nq, o, v), dtype=np.float32)
    b_oo = np.empty((nq, o, o), dtype=np.float32)
    b_vv = np.empty((nq, v, v), dtype=np.float32)
    for q in range(nq):
        b_ov[q] = gen_b_ov(shape, seed, q)
        b_oo[q] = gen_b_oo(shape, seed, q)
        b_vv[q] = gen_b_vv(shape, seed, q)
    return Problem(shape, seed, e_occ, e_virt, b_ov, b_oo, b_vv, gen_mu(shape, seed))


def factor_bits_range(shape: Shape, seed: int, q0: int, q1: int, pool=None):
    """The BF16-stored factors of Q = q0..q1-1 (the same values as make_problem) as uint16 bit
    patterns: (b_ov [n][o][v], b_oo [n][o][o], b_vv [n][v][v]).  Q values are drawn in parallel
    when a concurrent.futures executor is given (each Q has its own stream)."""
    if shape.storage != "bf16":
        raise ValueError("factor_bits_range is for BF16 storage")
    n, o, v = q1 - q0, shape.o, shape.v
    out = (np.empty((n, o, v), np.uint16), np.empty((n, o, o), np.uint16), np.empty((n, v, v), np.uint16))

    def one(q):
        k = q - q0
        out[0][k] = bf16_bits(gen_b_ov(shape, seed, q))
        out[1][k] = bf16_bits(gen_b_oo(shape, seed, q))
        out[2][k] = bf16_bits(gen_b_vv(shape, seed, q))

    if pool is None:
        for q in range(q0, q1):
            one(q)
    else:
        list(pool.map(one, range(q0, q1)))
    return out


def upload_factors_streamed(shape: Shape, seed: int, device: str = "cuda:0", threads: int = 16, q_chunk: int = 64,
                            progress=None):
    """Device tensors of a BF16-stored problem too large to hold on the host in FP32 (the o240
    shape's factors take 37 GB): the factors of make_problem drawn on the host a range of Q at a
    time (threads in parallel) and copied to the device as BF16.  Returns the dict of
    make_device_tensors (e_occ, e_virt, b_ov, b_oo, b_vv, mu), with exactly make_problem's values."""
    import concurrent.futures as cf

    import torch

    o, v, nq = shape.o, shape.v, shape.nq
    e_occ, e_virt = gen_energies(shape, seed)
    out = {"e_occ": torch.from_numpy(e_occ).to(device), "e_virt": torch.from_numpy(e_virt).to(device),
           "mu": torch.from_numpy(gen_mu(shape, seed)).to(device)}
    dev = [torch.empty((nq, o, v), dtype=torch.bfloat16, device=device),
           torch.empty((nq, o, o), dtype=torch.bfloat16, device=device),
           torch.empty((nq, v, v), dtype=torch.bfloat16, device=device)]
    with cf.ThreadPoolExecutor(max_workers=threads) as pool:
        for q0 in range(0, nq, q_chunk):
            q1 = min(nq, q0 + q_chunk)
            bits = factor_bits_range(shape, seed, q0, q1, pool)
            for t, b in zip(dev, bits):
                t[q0:q1].view(torch.int16).copy_(torch.from_numpy(b.view(np.int16)))
            if progress is not None:
                progress(q1)
    out.update(b_ov=dev[0], b_oo=dev[1], b_vv=dev[2])
    return out


def random_state(o: int, v: int, nrhs: int, seed: int, c0_scale: float = 1.0, c_scale: float = 1.0):
    """Random complex amplitudes for sigma-vector tests: c0 (nrhs,), c (nrhs, o, v)."""
    rng = _rng(seed, 100, nrhs)
    c0 = (rng.standard_normal(nrhs) + 1j * rng.standard_normal(nrhs)) * c0_scale
    c = (rng.standard_normal((nrhs, o, v)) + 1j * rng.standard_normal((nrhs, o, v))) * c_scale
    return c0.astype(np.complex128), c.astype(np.complex128)


# --------------------------------------------------------------------------------------
# The five workloads (shapes, pulses, time steps).
# --------------------------------------------------------------------------------------
KAPPA = 1e-4
AXES = ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))


@dataclass
class Workload:
    name: str
    shape: Shape
    seed: int
    dt: float
    n_steps: int
    pulses: List[Pulse] = field(default_factory=list)
    precision: str = "fp32"  # "fp32" | "mixed"


def kick_pulses(axes=AXES, kappa: float = KAPPA, exact: bool = False) -> List[Pulse]:
    return [Pulse(kind=PULSE_DELTA_EXACT if exact else PULSE_DELTA, e0=kappa, direction=tuple(a)) for a in axes]


def gauss_cos_scan(omega_low: float, e0: float, n: int = 64, fwhm: float = 400.0, t0: float = 400.0,
                   lo: float = 0.5, hi: float = 1.2) -> List[Pulse]:
    """Gaussian-envelope cosine pulses along z, carriers spanning [lo, hi] x omega_low."""
    out = []
    for r in range(n):
        w = omega_low * (lo + (hi - lo) * r / max(n - 1, 1))
        out.append(Pulse(kind=PULSE_GAUSS, e0=e0, omega=w, t0=t0, fwhm=fwhm, phase=math.pi / 2,
                         direction=(0.0, 0.0, 1.0)))
    return out


def workload(k: int) -> Workload:
    """k = 1..4: the single-molecule workloads (5 is the serving stream, see serving_requests)."""
    seed = SEED_BASE + k
    if k == 1:
        return Workload("o10_v40_nq120_kick_z", Shape(10, 40, 120, 0.05), seed, 0.05, 2000,
                        kick_pulses(axes=(AXES[2],)))
    if k == 2:
        return Workload("o60_v400_nq1500_kick_xyz", Shape(60, 400, 1500, 0.05), seed, 0.05, 20000,
                        kick_pulses())
    if k == 3:
        return Workload("o240_v1800_nq5000_kick_xyz_mixed", Shape(240, 1800, 5000, 0.02, storage="bf16"),
                        seed, 0.1, 4000, kick_pulses(), precision="mixed")
    if k == 4:
        # omega_low (lowest eigenvalue of A) is filled in by the caller that knows it
        return Workload("o40_v300_nq1000_gauss_cos_scan64", Shape(40, 300, 1000, 0.05), seed, 0.05, 16000, [])
    raise ValueError(k)


@dataclass
class Request:
    rid: int
    arrival: float
    shape: Shape
    seed: int
    n_steps: int
    dt: float
    pulse: Pulse


def serving_requests(n: int, rate: float = 20.0, seed: int = SEED_BASE + 5, o_min: int = 10,
                     o_max: int = 240) -> List[Request]:
    """Poisson arrivals of mixed-size requests: o ~ U{o_min..o_max}, v = floor(7.5 o),
    N_Q = 20 o, steps ~ U{500..8000}, dt 0.05, half delta kicks (z) and half Gaussian-sine
    pulses with E0 ~ U[0.001, 0.03], omega ~ U[0.3, 0.8], FWHM 400 au, t0 = half the run."""
    rng = _rng(seed, TENSOR_PULSE, 0)
    t = 0.0
    out = []
    for rid in range(n):
        t += rng.exponential(1.0 / rate)
        o = int(rng.integers(o_min, o_max + 1))
        v = int(math.floor(7.5 * o))
        steps = int(rng.integers(500, 8001))
        dt = 0.05
        if rng.uniform() < 0.5:
            p = Pulse(kind=PULSE_DELTA, e0=KAPPA, direction=(0.0, 0.0, 1.0))
        else:
            p = Pulse(kind=PULSE_GAUSS, e0=float(rng.uniform(0.001, 0.03)), omega=float(rng.uniform(0.3, 0.8)),
                      t0=0.5 * steps * dt, fwhm=400.0, direction=(0.0, 0.0, 1.0))
        out.append(Request(rid, t, Shape(o, v, 20 * o, 0.02, storage="bf16"), seed * 1000 + rid, steps, dt, p))
    return out


# --------------------------------------------------------------------------------------
# Device-side generation for large requests (serving): torch's counter-based CUDA generator,
# one generator per (seed, tensor), drawn in Q chunks.  Same distributions and rounding rule
# as make_problem (N(0,1) * s_eff in FP32, symmetric upper triangle mirrored, rounded to the
# storage dtype); the values differ from make_problem's host streams.
# --------------------------------------------------------------------------------------
def make_device_tensors(shape: Shape, seed: int, device: str = "cuda:0", q_chunk: int = 64):
    """Returns dict of device tensors e_occ, e_virt (f64), b_ov, b_oo, b_vv (f32 or bf16), mu (f64)."""
    import torch

    dt = torch.float32 if shape.storage == "f32" else torch.bfloat16
    o, v, nq = shape.o, shape.v, shape.nq
    s = float(np.float32(shape.s_eff))

    def gen(tensor):
        g = torch.Generator(device=device)
        g.manual_seed((int(seed) * 7919 + int(tensor)) % (2 ** 63))
        return g

    e_occ, e_virt = gen_energies(shape, seed)
    out = {"e_occ": torch.from_numpy(e_occ).to(device), "e_virt": torch.from_numpy(e_virt).to(device),
           "mu": torch.from_numpy(gen_mu(shape, seed)).to(device)}
    b_ov = torch.empty((nq, o, v), dtype=dt, device=device)
    b_oo = torch.empty((nq, o, o), dtype=dt, device=device)
    b_vv = torch.empty((nq, v, v), dtype=dt, device=device)
    g_ov, g_oo, g_vv = gen(TENSOR_B_OV), gen(TENSOR_B_OO), gen(TENSOR_B_VV)
    for q0 in range(0, nq, q_chunk):
        q1 = min(nq, q0 + q_chunk)
        n = q1 - q0
        b_ov[q0:q1] = (torch.randn((n, o, v), generator=g_ov, device=device) * s).to(dt)
        m = torch.randn((n, o, o), generator=g_oo, device=device)
        b_oo[q0:q1] = ((torch.triu(m) + torch.triu(m, 1).transpose(1, 2)) * s).to(dt)
        m = torch.randn((n, v, v), generator=g_vv, device=device)
        b_vv[q0:q1] = ((torch.triu(m) + torch.triu(m, 1).transpose(1, 2)) * s).to(dt)
        del m
    out.update(b_ov=b_ov, b_oo=b_oo, b_vv=b_vv)
    return out


def problem_from_device(shape: Shape, seed: int, t: dict) -> Problem:
    """Host copy (FP32 values) of device-generated tensors, for the oracle."""
    f = lambda x: x.float().cpu().numpy()  # noqa: E731
    return Problem(shape, seed, t["e_occ"].cpu().numpy(), t["e_virt"].cpu().numpy(), f(t["b_ov"]), f(t["b_oo"]),
                   f(t["b_vv"]), t["mu"].cpu().numpy())
