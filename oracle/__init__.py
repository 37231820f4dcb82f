"""Plain FP64 CPU oracle for RT-TDA (real-time Tamm-Dancoff) propagation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP implementation;
the only common module is the seeded input generator, which holds none of the
method's arithmetic.

Modules:
  rttda64   -- sigma vector, dipole coupling, pulses, RK4 propagation (direct
               density-fitted route) and the dense / eigenbasis route.
  spectrum  -- kick-spectrum post-processing of a dipole trace.
"""
