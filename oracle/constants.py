"""Physical constants used by the oracle.

The paper uses gamma_0, mu_0 and k_B without printing values (LLG equation,
Methods "Physics and discretization"; thermal-field sigma, Results "A
replica-batched engine").  Reading: the mumax3 gyromagnetic ratio (the paper
matches mumax3 conventions), the SI vacuum permeability 4*pi*1e-7 and the exact
SI Boltzmann constant; for the spin-transfer torque the exact SI reduced Planck
constant h / 2 pi and elementary charge.
"""
import math

GAMMA0 = 1.7595e11          # rad s^-1 T^-1
MU0 = 4.0e-7 * math.pi      # H/m
KB = 1.380649e-23           # J/K
HBAR = 6.62607015e-34 / (2.0 * math.pi)   # J s
QE = 1.602176634e-19        # C
