"""Closed forms of linear elastodynamics used to pin the CPU reference.

Each function states the textbook relation it evaluates; none of them shares
arithmetic with the lattice-Boltzmann code under test.
"""
import math

from scipy.optimize import brentq


def wave_speeds(lam, mu, rho=1.0):
    """Shear and dilatational wave speeds c_s = sqrt(mu/rho),
    c_d = sqrt((lambda + 2 mu)/rho) (paper, section 3 and section 5.1)."""
    return math.sqrt(mu / rho), math.sqrt((lam + 2 * mu) / rho)


def nu_from_speed_ratio(cd2_over_cs2):
    """Plane-strain Poisson ratio from c_d^2/c_s^2 = 2(1 - nu)/(1 - 2 nu)."""
    r = cd2_over_cs2
    return (r - 2.0) / (2.0 * (r - 1.0))


def freund_k0(t_star, nu, cd, t):
    """Mode-I stress intensity factor of a semi-infinite crack whose faces are
    suddenly loaded by a uniform traction t_star at t = 0, valid until waves
    from elsewhere arrive: K = 2 t* sqrt(1 - 2 nu)/(1 - nu) sqrt(c_d t/pi)
    (the paper's section 5.2, after Freund)."""
    return 2.0 * t_star * math.sqrt(1.0 - 2.0 * nu) / (1.0 - nu) * math.sqrt(cd * t / math.pi)


def rayleigh_speed(cs, cd):
    """Root c in (0, c_s) of (2 - c^2/c_s^2)^2 = 4 sqrt((1 - c^2/c_d^2)(1 - c^2/c_s^2))."""
    def f(c):
        a = c * c / (cs * cs)
        b = c * c / (cd * cd)
        return (2.0 - a) ** 2 - 4.0 * math.sqrt((1.0 - b) * (1.0 - a))
    return brentq(f, 1e-6 * cs, cs * (1 - 1e-12), xtol=1e-15)


def plane_strain_modulus(lam, mu):
    """Uniaxial-stress stiffness of a strip in plane strain with free lateral
    faces: E' = 4 mu (lambda + mu)/(lambda + 2 mu)."""
    return 4.0 * mu * (lam + mu) / (lam + 2.0 * mu)
