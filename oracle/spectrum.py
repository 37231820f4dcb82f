"""Kick-spectrum post-processing of a dipole trace (test harness; used on GPU and oracle traces alike).

Follows the paper's recipe (Absorption spectrum subsection and eq. fourier_transform):
a Hann window with mirroring -- read here as the half-Hann window on [0, T], which
equals a full Hann window on the odd (mirrored) record of length 2T --, zero padding
with 50 000 zeros, the Fourier transform, and a factor omega:

    S(omega) = omega * Im sum_n h_n (mu_n - mu_0) exp(i omega t_n) dt / kappa,
    h_n = (1 + cos(pi n / N)) / 2,  t_n = n dt,  n = 0..N.

For a first-order kick of strength kappa the induced dipole is
2 kappa sum_I |M_0I|^2 sin(w_I t), so S has peaks at the excitation energies with
heights proportional to w_I |M_0I|^2 (oscillator strengths).
Peaks: local maxima of at least `rel_height` of the largest, refined by 3-point
parabolic interpolation and optionally by maximising the un-gridded transform.
"""
from __future__ import annotations

import math

import numpy as np

HARTREE_EV = 27.211386
AU_FS = 0.02418884326585747


def window(n_samples: int) -> np.ndarray:
    N = n_samples - 1
    n = np.arange(n_samples)
    return 0.5 * (1.0 + np.cos(math.pi * n / max(N, 1)))


def kick_spectrum(trace, dt: float, kappa: float, n_pad: int = 50000):
    """Returns (omega grid [Ha], S(omega)) on the FFT grid 2 pi k / (M dt)."""
    trace = np.asarray(trace, dtype=np.float64)
    s = (trace - trace[0]) * window(trace.size)
    M = trace.size + n_pad
    F = np.fft.ifft(s, n=M) * M * dt  # sum_n s_n exp(+i 2 pi k n / M) dt
    omega = 2.0 * math.pi * np.arange(M) / (M * dt)
    half = M // 2
    return omega[:half], omega[:half] * F.imag[:half] / kappa


def dtft(trace, dt: float, kappa: float, omega: float) -> float:
    """S(omega) without the grid (same definition as kick_spectrum)."""
    trace = np.asarray(trace, dtype=np.float64)
    s = (trace - trace[0]) * window(trace.size)
    t = np.arange(trace.size) * dt
    return omega * float(np.dot(s, np.sin(omega * t))) * dt / kappa


def find_peaks(omega, S, rel_height: float = 0.05, omega_max: float = None):
    S = np.asarray(S)
    if omega_max is not None:
        keep = omega <= omega_max
        omega, S = omega[keep], S[keep]
    top = S.max()
    idx = np.where((S[1:-1] > S[:-2]) & (S[1:-1] >= S[2:]) & (S[1:-1] >= rel_height * top))[0] + 1
    out = []
    dw = omega[1] - omega[0]
    for k in idx:
        y0, y1, y2 = S[k - 1], S[k], S[k + 1]
        den = y0 - 2.0 * y1 + y2
        shift = 0.5 * (y0 - y2) / den if den != 0 else 0.0
        out.append((omega[k] + shift * dw, y1 - 0.25 * (y0 - y2) * shift))
    return out


def refine_peak(trace, dt: float, kappa: float, w_guess: float, half_width: float, tol: float = 1e-10) -> float:
    """Maximise the un-gridded transform on [w_guess - half_width, w_guess + half_width] (golden section)."""
    g = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = w_guess - half_width, w_guess + half_width
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = dtft(trace, dt, kappa, c), dtft(trace, dt, kappa, d)
    while b - a > tol:
        if fc > fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = dtft(trace, dt, kappa, c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = dtft(trace, dt, kappa, d)
    return 0.5 * (a + b)


def peaks(trace, dt: float, kappa: float, rel_height: float = 0.05, omega_max: float = None,
          refine: bool = False, n_pad: int = 50000):
    w, S = kick_spectrum(trace, dt, kappa, n_pad=n_pad)
    pk = find_peaks(w, S, rel_height=rel_height, omega_max=omega_max)
    if refine:
        dw = w[1] - w[0]
        pk = [(refine_peak(trace, dt, kappa, p, dw), h) for p, h in pk]
    return pk


def correlation_spectrum(corr, dt: float, omega) -> np.ndarray:
    """The spectrum of a time-correlation function (eq. time_correlation_function) by the paper's
    omega-weighted transform (eq. fourier_transform), with the same half-Hann window as the dipole
    spectrum:  R(omega) = omega Re sum_n h_n R_n exp(i omega t_n) dt  for each omega (un-gridded).
    For R_n = sum_I |y_I|^2 r_I^n with |r_I| = 1, r_I = exp(-i w_I dt), the terms peak at w_I."""
    corr = np.asarray(corr, dtype=np.complex128)
    omega = np.atleast_1d(np.asarray(omega, dtype=np.float64))
    s = corr * window(corr.size)
    t = np.arange(corr.size) * dt
    out = np.empty(omega.size)
    for k, om in enumerate(omega):
        out[k] = om * float(np.real(np.sum(s * np.exp(1j * om * t)))) * dt
    return out


def correlation_peaks(corr, dt: float, omega, rel_height: float = 0.05, refine: bool = True):
    """Local maxima of correlation_spectrum on the grid omega (at least rel_height of the largest),
    each refined by maximising the un-gridded transform within one grid step (golden section)."""
    omega = np.asarray(omega, dtype=np.float64)
    S = correlation_spectrum(corr, dt, omega)
    out = []
    for om, h in find_peaks(omega, S, rel_height=rel_height):
        if refine:
            g = (math.sqrt(5.0) - 1.0) / 2.0
            dw = omega[1] - omega[0]
            a, b = om - dw, om + dw
            c, d = b - g * (b - a), a + g * (b - a)
            fc, fd = correlation_spectrum(corr, dt, c)[0], correlation_spectrum(corr, dt, d)[0]
            while b - a > 1e-10:
                if fc > fd:
                    b, d, fd = d, c, fc
                    c = b - g * (b - a)
                    fc = correlation_spectrum(corr, dt, c)[0]
                else:
                    a, c, fc = c, d, fd
                    d = a + g * (b - a)
                    fd = correlation_spectrum(corr, dt, d)[0]
            om = 0.5 * (a + b)
            h = correlation_spectrum(corr, dt, om)[0]
        out.append((om, h))
    return out


def resolution(total_time_au: float) -> float:
    """Frequency resolution 2 pi / T in Ha."""
    return 2.0 * math.pi / total_time_au
