"""FP64 CPU oracle of the micropolar elastoplastic FFT-based basic scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP path; its only common
input is the seeded generator module `paper_2409_10774_amd.workloads`, which
holds none of the method's arithmetic.

Modules
  micropolar  Eqs. 6/8 stiffnesses, Alg. 1 radial return, the reference-medium
              Green operator (built from the balance laws Eqs. 1-2 and solved
              densely per frequency), error measure Eqs. 36-38, Alg. 2 driver.
  tangent     App. C continuum tangents and an RK4 integrator with yield-event
              location (independent route to the stresses for the pins).

Pins live in tests/test_oracle_*.py.
"""
