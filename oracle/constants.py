"""Physical constants of the oracle (kept separate from the GPU library's copies).

MU0       vacuum permeability, 4*pi*1e-7 T m / A (the classical SI value).
KB        Boltzmann constant in J/K.
GAMMA_LL  default gyromagnetic ratio of the Landau-Lifshitz equation in
          rad/(T s).  The paper leaves the default open (section "Landau-
          Lifshitz torque") but uses 1.7595e11 in its solver-convergence script
          (appendix, "Solver convergence and MaxErr") for the analytic period.
"""
import math

MU0 = 4.0e-7 * math.pi
GAMMA_LL = 1.7595e11
KB = 1.380649e-23  # Boltzmann constant, J/K (exact in the SI since 2019)
