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


def _freund_g(xi, a, b):
    """Phase of the Rayleigh function on the branch cut a < xi < b:
    tan g = 4 xi^2 sqrt((xi^2 - a^2)(b^2 - xi^2)) / (b^2 - 2 xi^2)^2, with
    g in [0, pi/2] (the arctan in the inner integral of eq:ki1)."""
    num = 4.0 * xi * xi * math.sqrt(max((xi * xi - a * a) * (b * b - xi * xi), 0.0))
    return math.atan2(num, (b * b - 2.0 * xi * xi) ** 2)


def _freund_inner(eta, a, b):
    """Real part of the inner integral of eq:ki1 divided by pi:
    (1/pi) p.v. int_a^b g(xi) 2 eta/(xi^2 - eta^2) dxi, written as the
    principal value of [g(xi) 2 eta/(xi + eta)]/(xi - eta)."""
    from scipy.integrate import quad
    f = lambda xi: _freund_g(xi, a, b) * 2.0 * eta / (xi + eta)
    if a < eta < b:
        v = quad(f, a, b, weight="cauchy", wvar=eta, limit=400)[0]
    else:
        v = quad(lambda xi: f(xi) / (xi - eta), a, b, limit=400)[0]
    return v / math.pi


def _freund_outer(T, a, b, cr, inner):
    """int_a^T Im(...) d eta of eq:ki1 (slownesses, l_c = 1 in T = t/l_c).

    The inner path passes xi = eta (for a < eta < b) on a small semicircle
    above the real axis, which adds -i pi times the residue g(eta) to the
    principal value; after the 1/pi the exponential carries the phase
    e^{-i g(eta)}.  sqrt((a - eta)/(a + eta)) = i sqrt((eta - a)/(eta + a))
    for eta > a (principal branch).  Every other factor is real, so
    Im(i e^{-i g} X) = X cos g.  The pole of (c_r + eta)/(c_r - eta) at
    eta = c_r is taken as a principal value."""
    from scipy.integrate import quad

    def h(eta):
        ph = math.cos(_freund_g(eta, a, b)) if a < eta < b else 1.0
        return (math.sqrt(max(T - eta, 0.0)) * math.sqrt(max(eta - a, 0.0) / (eta + a)) * (cr + eta) / eta
                * math.exp(inner(eta)) * ph)

    if T > cr:
        # int h/(c_r - eta) = -p.v. int h/(eta - c_r)
        return -quad(h, a, T, weight="cauchy", wvar=cr, limit=400)[0]
    return quad(lambda e: h(e) / (cr - e), a, T, limit=400)[0]


def freund_k1(t_star, nu, cd, cs, lc, t, f_plus0=0.8774):
    """Mode-I stress intensity factor at one tip of a crack of length lc whose
    faces are suddenly loaded by t_star, from t = lc/c_d (when the waves
    scattered by the other tip arrive) to 2 lc/c_d: K^0 plus Freund's
    correction (the paper's eq:ki1, section 5.2), with slownesses a = 1/c_d,
    b = 1/c_s and c_r = 1/c_R, and F_+(0) as the paper gives it.  The
    contour and branch choices are those of :func:`_freund_outer`."""
    k0 = freund_k0(t_star, nu, cd, t)
    a, b = 1.0 / cd, 1.0 / cs
    cr = 1.0 / rayleigh_speed(cs, cd)
    T = t / lc
    if T <= a:
        return k0
    I = _freund_outer(T, a, b, cr, lambda eta: _freund_inner(eta, a, b))
    return k0 + 2.0 * t_star * f_plus0 / math.pi * math.sqrt(2.0 * lc / math.pi) * I


def freund_k1_curve(t_star, nu, cd, cs, lc, times, f_plus0=0.8774, nodes=2400):
    """freund_k1 at many times: the inner integral (a smooth function of eta
    on [a, 2.5 a] apart from square-root behaviour at b) is tabulated once on
    `nodes` points that include b and interpolated by cubic splines on each
    side of b.  Valid for t <= 2.5 lc/c_d."""
    import numpy as np
    from scipy.interpolate import CubicSpline

    a, b = 1.0 / cd, 1.0 / cs
    cr = 1.0 / rayleigh_speed(cs, cd)
    lo = np.linspace(a, b, nodes // 2)
    hi = np.linspace(b, 2.5 * a, nodes // 2)
    s_lo = CubicSpline(lo, [_freund_inner(e, a, b) for e in lo])
    s_hi = CubicSpline(hi, [_freund_inner(e, a, b) for e in hi])
    inner = lambda eta: float(s_lo(eta) if eta <= b else s_hi(eta))
    out = []
    for t in times:
        k0 = freund_k0(t_star, nu, cd, max(t, 0.0))
        T = t / lc
        if T <= a:
            out.append(k0)
            continue
        if T > 2.5 * a:
            raise ValueError("freund_k1_curve is tabulated up to t = 2.5 lc/c_d")
        I = _freund_outer(T, a, b, cr, inner)
        out.append(k0 + 2.0 * t_star * f_plus0 / math.pi * math.sqrt(2.0 * lc / math.pi) * I)
    return np.array(out)
