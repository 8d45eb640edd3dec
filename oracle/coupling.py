"""TEST INFRASTRUCTURE ONLY: the coupling of the gravity solve to the
hydrodynamic update, written out from its definitions (numpy, FP64).

Sec. 2.3, source vector S (right-hand sides of the momentum and energy
equations of Sec. 2.1):
    S_s = rho g + Omega x s
    S_E = 1/2 (phi drho/dt - rho dphi/dt) + rho Omega . (x x g)
(the paper's energy entry is printed as a cross product; the energy equation
it comes from has the scalar rho Omega . (x x g), which is what is used here)
and, after each potential solve, E_after = E_before + 1/2 rho (phi_before -
phi_after).
"""
import numpy as np


def gravity_sources(omega, x, rho, s, phi, g, drho_dt=None, dphi_dt=None):
    """x, s, g: (3, n); rho, phi, drho_dt, dphi_dt: (n,).  Returns (S_s (3, n), S_E (n,))."""
    omega = np.asarray(omega, dtype=np.float64)
    drho_dt = np.zeros_like(rho) if drho_dt is None else drho_dt
    dphi_dt = np.zeros_like(rho) if dphi_dt is None else dphi_dt
    om = omega[:, None]
    S_s = rho[None, :] * g + np.cross(om, s, axis=0)
    x_cross_g = np.cross(x, g, axis=0)
    S_E = 0.5 * (phi * drho_dt - rho * dphi_dt) + rho * (om * x_cross_g).sum(axis=0)
    return S_s, S_E


def energy_update(E, rho, phi_before, phi_after):
    return E + 0.5 * rho * (phi_before - phi_after)
