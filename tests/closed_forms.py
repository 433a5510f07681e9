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


def freund_k1(t_star, nu, cd, cs, lc, t, f_plus0=0.8774):
    """Mode-I stress intensity factor at one tip of a crack of length lc whose
    faces are suddenly loaded by t_star, from t = lc/c_d (when the waves
    scattered by the other tip arrive) to 2 lc/c_d: K^0 plus Freund's
    correction (the paper's eq:ki1), with slownesses a = 1/c_d, b = 1/c_s and
    c_r = 1/c_R.  Both integrals are Cauchy principal values: the inner one
    at xi = eta, the outer one at eta = c_r; each is written as
    p.v. int f(x)/(x - c) dx and evaluated by quadrature with that weight."""
    import numpy as np
    from scipy.integrate import quad

    k0 = freund_k0(t_star, nu, cd, t)
    a, b = 1.0 / cd, 1.0 / cs
    cr = 1.0 / rayleigh_speed(cs, cd)
    T = t / lc
    if T <= a:
        return k0

    def g(xi):
        num = 4.0 * xi * xi * math.sqrt(max((xi * xi - a * a) * (b * b - xi * xi), 0.0))
        den = (b * b - 2.0 * xi * xi) ** 2
        return math.atan2(num, den)

    def inner(eta):
        # (1/pi) p.v. int_a^b g(xi) 2 eta / (xi^2 - eta^2) dxi
        f = lambda xi: g(xi) * 2.0 * eta / (xi + eta)
        if a < eta < b:
            v = quad(f, a, b, weight="cauchy", wvar=eta, limit=400)[0]
        else:
            v = quad(lambda xi: f(xi) / (xi - eta), a, b, limit=400)[0]
        return v / math.pi

    def h(eta):
        # Im of the outer integrand times (c_r - eta): sqrt((a - eta)/(a + eta))
        # is i sqrt((eta - a)/(eta + a)) for eta > a, everything else is real
        return (math.sqrt(max(T - eta, 0.0)) * math.sqrt(max(eta - a, 0.0) / (eta + a)) * (cr + eta) / eta
                * math.exp(inner(eta)))

    if T > cr:
        # int h/(c_r - eta) = -p.v. int h/(eta - c_r)
        integral = -quad(h, a, T, weight="cauchy", wvar=cr, limit=400)[0]
    else:
        integral = quad(lambda e: h(e) / (cr - e), a, T, limit=400)[0]
    return k0 + 2.0 * t_star * f_plus0 / math.pi * math.sqrt(2.0 * lc / math.pi) * integral
