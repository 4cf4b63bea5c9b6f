"""Cross sections used by the oracle.

Discharge (Sec. IV.A, 'Particle Collisions'): the paper tabulates LXcat data,
which is not available here; the workloads use analytic forms instead:
  e-Ar elastic      sigma_el (constant)
  e-Ar excitation   sigma0_exc * ln(x)/x, x = eps/E_exc, zero for x <= 1
  e-Ar ionisation   sigma0_ion * ln(x)/x, x = eps/E_ion, zero for x <= 1
  Ar+-Ar resonant charge exchange   sigma_cx (constant)
eps is the interaction energy 0.5 * m_r * v_r^2 in eV (Sec. IV.A).

Test particles (Sec. IV.B, 'Binary Interactions'): variable hard sphere,
total cross section sigma_T = pi * b_max^2 with b_max from Eq. (8).
"""
import math
import numpy as np

from . import constants as C


def ln_x_over_x(eps_ev, e_th, sigma0):
    """sigma0 * ln(x)/x above threshold x = eps/E_th > 1, else 0 (threshold check of Eq. (6))."""
    eps_ev = np.asarray(eps_ev, dtype=np.float64)
    x = eps_ev / e_th
    with np.errstate(divide="ignore", invalid="ignore"):
        s = sigma0 * np.log(x) / x
    return np.where(x > 1.0, s, 0.0)


def electron_sigmas(eps_ev, xs):
    """(sigma_el, sigma_exc, sigma_ion) in m^2, the fixed process order of the selection."""
    eps_ev = np.asarray(eps_ev, dtype=np.float64)
    s_el = np.full_like(eps_ev, xs["sigma_el"])
    s_exc = ln_x_over_x(eps_ev, xs["eth_exc"], xs["sigma0_exc"])
    s_ion = ln_x_over_x(eps_ev, xs["eth_ion"], xs["sigma0_ion"])
    return s_el, s_exc, s_ion


def vhs_bmax(v_r, m_r, d_ref, omega, t_ref):
    """Maximum impact parameter of the VHS model, Eq. (8)."""
    v_r = np.asarray(v_r, dtype=np.float64)
    with np.errstate(divide="ignore"):
        arg = (2.0 * C.K_B * t_ref / (m_r * v_r ** 2)) ** (omega - 0.5)
    return d_ref * np.sqrt(arg / math.gamma(2.5 - omega))


def vhs_sigma(v_r, m_r, d_ref, omega, t_ref):
    """VHS total cross section sigma_T = pi b_max^2 (Sec. IV.B)."""
    return math.pi * vhs_bmax(v_r, m_r, d_ref, omega, t_ref) ** 2
