"""Reference oracle for the micromagnetic effective-field / torque hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, double-precision
CPU implementation of what the GPU library computes, written from the MuMax3
paper (Vansteenkiste et al., "The design and verification of MuMax3",
arXiv:1406.7635).  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path (the HIP library and its
Python binding) never does, and this package imports nothing from the product.

Modules
-------
constants   physical constants used by the oracle (its own copies)
demag       Newell demagnetising tensor, far-field quadrature, FFT and direct
            convolution, periodic images (paper section "Magnetostatic field")
fields      exchange, uniaxial anisotropy, Zeeman, effective field, Landau-
            Lifshitz torque and energies (sections "Landau-Lifshitz torque",
            "Heisenberg exchange interaction", "Magneto-crystalline anisotropy")
integrate   classical RK4, Heun 2(1), Bogacki-Shampine 3(2), Dormand-Prince 5(4), the
            adaptive step controller and relax() (sections "Dynamics",
            "Adaptive time step", "Energy minimization")
thermal     Brown's thermal field with a counter-based Philox4x32-10 generator,
            Heun steps at finite temperature (section "Thermal fluctuations")

Parity status: every function is pinned by the `-m "not gpu"` tests in
tests/test_oracle_*.py against closed forms, brute force or invariants, except
where a function's docstring says "parity unpinned".
"""
