"""Physical constants used by the oracle.

The paper uses gamma_0, mu_0 and k_B without printing values (LLG equation,
Methods "Physics and discretization"; thermal-field sigma, Results "A
replica-batched engine").  Reading: the mumax3 gyromagnetic ratio (the paper
matches mumax3 conventions), the SI vacuum permeability 4*pi*1e-7 and the exact
SI Boltzmann constant.
"""
import math

GAMMA0 = 1.7595e11          # rad s^-1 T^-1
MU0 = 4.0e-7 * math.pi      # H/m
KB = 1.380649e-23           # J/K
