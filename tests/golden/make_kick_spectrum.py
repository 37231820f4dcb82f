"""Writes the oracle's kick-spectrum peaks of a workload to tests/golden/<name>_kick_peaks.txt.

Calls only the FP64 oracle and the seeded input generator.  Route: dense A (explicit DF
sums), eigh, and the first-order (linear in kappa) dipole trace of the exact RK4 map in the
eigenbasis (oracle.rttda64.linear_kick_trace), which is the full trace minus its O(kappa^2)
part (a smooth background that moves peak positions by far less than 1e-6 Ha).  Peaks come from
oracle.spectrum (same post-processing as applied to GPU traces).

    python tests/golden/make_kick_spectrum.py cfg2
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import rttda64 as O  # noqa: E402
from oracle import spectrum as S  # noqa: E402
from paper_2601_16949_amd import inputs as I  # noqa: E402


def main(name):
    k = {"cfg1": 1, "cfg2": 2}[name]
    wl = I.workload(k)
    t0 = time.time()
    prob = I.make_problem(wl.shape, wl.seed)
    op = O.Operator.from_problem(prob)
    A = O.dense_A_blas(op)
    print(f"dense A {A.shape} in {time.time() - t0:.0f} s", flush=True)
    w, U = np.linalg.eigh(A)
    del A
    print(f"eigh in {time.time() - t0:.0f} s", flush=True)
    lines = [f"# oracle kick-spectrum peaks of {wl.name} (dt {wl.dt}, {wl.n_steps} steps, kappa {I.KAPPA})",
             "# written by tests/golden/make_kick_spectrum.py (FP64 oracle: eigh + exact RK4 map, linear in kappa)",
             f"# lowest eigenvalue {w[0]:.12f} Ha, highest {w[-1]:.12f} Ha",
             "# columns: direction index, peak omega (Ha), peak height"]
    for r, p in enumerate(wl.pulses):
        _, mov, _ = O.dipole_blocks(op, p.direction)
        z = U.T @ (np.sqrt(2.0) * mov.reshape(-1))
        tr = O.linear_kick_trace(w, z, p.e0, wl.dt, wl.n_steps)
        pk = S.peaks(tr, wl.dt, p.e0, rel_height=0.05, omega_max=8.0)
        for om, h in pk:
            lines.append(f"{r} {om:.10f} {h:.6e}")
        print(f"direction {r}: {len(pk)} peaks", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_kick_peaks.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {path} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "cfg2")
