"""Physical constants (CODATA 2018) and species data used by the oracle.

The paper fixes no constant set; CODATA 2018 is taken (e and k_B are exact in
SI since 2019).  The argon density of the paper's example (Sec. III, 0.5 Pa at
650 K, about 5.57e13 cm^-3) follows from n = p / (k_B T) with these values and
pins ``gas_density``.
"""

E_CHARGE = 1.602176634e-19      # C, exact
K_B = 1.380649e-23              # J/K, exact
M_E = 9.1093837015e-31          # kg
EPS0 = 8.8541878128e-12         # F/m
AMU = 1.66053906660e-27         # kg
M_AR = 39.948 * AMU             # argon atom / Ar+ ion (electron mass neglected)
M_AL = 26.9815385 * AMU         # aluminium atom


def gas_density(p_pa, t_k):
    """Ideal-gas background density n = p / (k_B T) in m^-3 (Sec. III)."""
    return p_pa / (K_B * t_k)
