"""Growth rates of small disturbances in a strip between two traction-free
walls, from an independent linearisation of one time step.

The strip is periodic in x; its rows y = 0..H-1 are material, and the two
walls cross the links that leave the strip at fraction q of their length
(the bottom wall at y = -q, the top one at y = H - 1 + q), the same q for
every cut link, so the geometry does not depend on x.  A disturbance of the
rest state proportional to exp(i k x) therefore stays one, and one time step
maps its nine complex population amplitudes per row linearly onto the next
ones.  This module builds that map row by row, in plain loops, directly from
the paper's equations, and returns the largest modulus of its eigenvalues:
the growth factor per step of the fastest mode of wave number k.

What the step does (deviations from rest; lattice units, c_s^2 = 1/3,
closure with the populations' own second moment):

* section 3, eq:moments: the density, momentum and second moment of the
  populations of each row;
* eq:sourceterm: S = ((mu - lambda)/rho) grad rho, linearised about rho = 1,
  with the isotropic D2Q9 gradient 3 sum_i w_i c_i rho(x + c_i); across a
  cut link the neighbour's density is extrapolated from the opposite side,
  2 rho(x) - rho(x - c_i);
* eq:fieq and eq:coll: BGK relaxation toward the equilibrium of (rho, j + S/2,
  P) with the forcing term (1 - 1/(2 tau)) w_i c_i.S / c_s^2;
* eq:stream: every population moves along its link; a population that would
  arrive from outside the strip comes from the Neumann rule on the cut link
  instead -- section 4.2, eq:abbnoncon (eq:abbcon at q = 1/2), with the
  boundary density and stress of eq:bcchainneum and eq:trafocauchy for a
  traction-free wall: the boundary Cauchy stress is sigma_tt e_t e_t, and
  the boundary Poisson stress -sigma* + (lambda - mu)(1 - rho_bd) I.  With the
  paper's rule (order 1) rho_bd and sigma_tt are extrapolated linearly
  along the link, (1 + q) v(x) - q v(x - c); with order 0 they are taken at
  the boundary site.

Nothing here is shared with the CPU reference or the GPU kernels.
"""
import cmath
import math

import numpy as np

C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
BACK = [0, 3, 4, 1, 2, 7, 8, 5, 6]
W = [4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4


def _double_dot(A, c):
    """A:(c c - I/3) for a symmetric 2x2 tensor A = (Axx, Ayy, Axy)."""
    axx, ayy, axy = A
    cx, cy = c
    return axx * cx * cx + ayy * cy * cy + 2.0 * axy * cx * cy - (axx + ayy) / 3.0


def _equilibrium_deviation(i, drho, jx, jy, P):
    """f_eq,i(1 + drho, j, P) - f_eq,i(1, 0, 0) from eq:fieq:
    w_i (rho + c.j/c_s^2 + (P - rho c_s^2 I):(c c - c_s^2 I)/(2 c_s^4))."""
    cx, cy = C[i]
    rho_term = drho
    j_term = 3.0 * (cx * jx + cy * jy)
    iso = -drho / 3.0                                  # the change of -rho c_s^2 I
    stress = 4.5 * _double_dot((P[0] + iso, P[1] + iso, P[2]), C[i])
    return W[i] * (rho_term + j_term + stress)


def step_operator(H, k, lam, mu, tau, q, order):
    """The matrix (9H x 9H, complex) of one step acting on the amplitudes
    f[i, y] (index i*H + y) of a disturbance exp(i k x); lam, mu in lattice
    units (mu = 1/3)."""
    n = 9 * H
    basis = np.eye(n, dtype=complex)
    f = {(i, y): basis[i * H + y] for i in range(9) for y in range(H)}   # each a row of the identity
    shift = [cmath.exp(1j * k * C[i][0]) for i in range(9)]              # value at x + c_i relative to x

    inside = lambda y: 0 <= y < H                                          # noqa: E731
    # moments of every row (eq:moments)
    rho, jx, jy, P = {}, {}, {}, {}
    for y in range(H):
        rho[y] = sum(f[(i, y)] for i in range(9))
        jx[y] = sum(C[i][0] * f[(i, y)] for i in range(9))
        jy[y] = sum(C[i][1] * f[(i, y)] for i in range(9))
        P[y] = (sum(C[i][0] ** 2 * f[(i, y)] for i in range(9)),
                sum(C[i][1] ** 2 * f[(i, y)] for i in range(9)),
                sum(C[i][0] * C[i][1] * f[(i, y)] for i in range(9)))
    # density of the neighbour across link i, extrapolated across cut links
    def rho_across(y, i):
        yy = y + C[i][1]
        if inside(yy):
            return rho[y + C[i][1]] * shift[i]
        yb = y - C[i][1]
        if inside(yb):
            return 2.0 * rho[y] - rho[yb] * shift[BACK[i]]
        return rho[y]
    # collision (eq:coll with eq:sourceterm)
    fcol = {}
    for y in range(H):
        gx = 3.0 * sum(W[i] * C[i][0] * rho_across(y, i) for i in range(1, 9))
        gy = 3.0 * sum(W[i] * C[i][1] * rho_across(y, i) for i in range(1, 9))
        Sx, Sy = (mu - lam) * gx, (mu - lam) * gy
        ux, uy = jx[y] + 0.5 * Sx, jy[y] + 0.5 * Sy
        for i in range(9):
            feq = _equilibrium_deviation(i, rho[y], ux, uy, P[y])
            psi = 3.0 * W[i] * (C[i][0] * Sx + C[i][1] * Sy)
            fcol[(i, y)] = f[(i, y)] - (f[(i, y)] - feq) / tau + (1.0 - 0.5 / tau) * psi
    # Cauchy stress of a row, from the Poisson stress and eq:approxdiv:
    # sigma = -P + (lambda - mu)(1 - rho) I; on a horizontal wall the
    # tangential direction is x, so sigma_tt = sigma_xx
    sigma_tt = {y: -P[y][0] - (lam - mu) * rho[y] for y in range(H)}
    kappa = (1.0 - 2.0 * q) / (1.0 + 2.0 * q)
    beta = 2.0 / (1.0 + 2.0 * q)
    new = {}
    for y in range(H):
        for i in range(9):
            src = y - C[i][1]
            if inside(src):
                new[(i, y)] = fcol[(i, src)] * shift[BACK[i]]
                continue
            # the link (x, k), k = BACK[i], leaves the strip: eq:abbnoncon
            kk = BACK[i]
            yin = y - C[kk][1]                          # row of x - c_k (inside the strip)
            back = shift[BACK[kk]]                      # x - c_k lies at column offset -c_k,x
            if order == 1:
                drho_bd = (1.0 + q) * rho[y] - q * rho[yin] * back
                stt = (1.0 + q) * sigma_tt[y] - q * sigma_tt[yin] * back
            else:
                drho_bd = rho[y]
                stt = sigma_tt[y]
            # boundary Cauchy stress sigma_tt e_t e_t (e_t = +-x), Poisson stress (eq:bcchainneum)
            Pstar = (-stt - (lam - mu) * drho_bd, -(lam - mu) * drho_bd, 0.0 * stt)
            E = 2.0 * _equilibrium_deviation(kk, drho_bd, 0.0, 0.0, Pstar)
            new[(i, y)] = -fcol[(kk, y)] - kappa * (fcol[(kk, yin)] * back + fcol[(i, y)]) + beta * E
    A = np.zeros((n, n), dtype=complex)
    for (i, y), v in new.items():
        A[i * H + y] = v
    return A


def max_growth(H, nx, lam_over_mu, tau, q, order):
    """Largest eigenvalue modulus of the one-step map over the wave numbers
    2 pi m / nx of a strip nx columns wide."""
    mu = 1.0 / 3.0
    lam = lam_over_mu * mu
    worst = 0.0
    for m in range(nx // 2 + 1):
        A = step_operator(H, 2.0 * math.pi * m / nx, lam, mu, tau, q, order)
        worst = max(worst, float(np.abs(np.linalg.eigvals(A)).max()))
    return worst
