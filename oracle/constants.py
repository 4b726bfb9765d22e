"""CODATA 2022 physical constants (SI), as published by NIST.

Test infrastructure only (see the package docstring).
"""

E_CHARGE = 1.602176634e-19          # elementary charge, C (exact)
M_E = 9.1093837139e-31              # electron mass, kg
EPS0 = 8.8541878188e-12             # vacuum permittivity, F/m
K_B = 1.380649e-23                  # Boltzmann constant, J/K (exact)
AMU = 1.66053906892e-27             # atomic mass constant, kg
H_PLANCK = 6.62607015e-34           # Planck constant, J s (exact)

M_CU_AMU = 63.546                   # Cu standard atomic weight
M_CU = M_CU_AMU * AMU               # Cu atom and Cu+ ion mass (electron mass
                                    # of the ion neglected), kg

TWO_PI = 6.283185307179586          # 2*pi rounded to binary64
E_EULER = 2.718281828459045         # e rounded to binary64

# Species indices: electron, Cu atom, Cu+ and Cu2+ (a higher charge state
# made by electron-impact ionisation of Cu+).
ELECTRON, NEUTRAL, ION, ION2 = 0, 1, 2, 3
NSPECIES = 4
CHARGE_SIGN = (-1, 0, +1, +2)
MASS = (M_E, M_CU, M_CU, M_CU)
