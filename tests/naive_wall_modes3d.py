"""Growth rates of small disturbances in a three-dimensional slab between two
traction-free walls, from an independent linearisation of one D3Q19 time
step.

The slab's sites x = 0..H-1 are material and it is periodic in y and z; the
two walls cross the links that leave it at fraction q of their length (at
x = -q and x = H - 1 + q), the same q for every cut link.  A disturbance of
the rest state proportional to exp(i (k_y y + k_z z)) stays one, and one
step maps its 19 complex population amplitudes per plane x linearly onto the
next ones.  This module builds that map plane by plane, in plain loops, from
the equations, and returns the largest modulus of its eigenvalues.

What the step does (deviations from rest; lattice units, c_s^2 = 1/3,
weights 1/3, 1/18, 1/36; the populations' own second moment in the
equilibrium):

* section 3, eq:moments: density, momentum and second moment per plane;
* eq:sourceterm: S = ((mu - lambda)/rho) grad rho linearised about rho = 1,
  with the isotropic gradient 3 sum_i w_i c_i rho(x + c_i); across a cut
  link the neighbour's density is 2 rho(x) - rho(x - c_i), or rho(x) when
  that is cut as well;
* eq:fieq and eq:coll: BGK relaxation toward the equilibrium of (rho,
  j + S/2, P) with the forcing term (1 - 1/(2 tau)) 3 w_i c_i.S;
* eq:stream: a population that would arrive from beyond a wall comes from
  the Neumann rule on the cut link instead (eq:abbnoncon, eq:abbcon at
  q = 1/2), with the boundary Cauchy stress of a traction-free wall with
  normal n = -+x: sigma* = Pi sigma_b Pi, Pi = I - n n (its normal row is
  the zero traction, its tangential block the material's), and the boundary
  Poisson stress -sigma* - (lambda - mu) drho_bd I; sigma_b and drho_bd are
  taken at the boundary site (order 0) or extrapolated along the link,
  (1 + q) v(x) - q v(x - c) (order 1).

Nothing here is shared with the CPU reference or the GPU kernels.
"""
import cmath
import itertools
import math

import numpy as np

# D3Q19 velocities (any order serves: the map's spectrum does not depend on it)
C = [(0, 0, 0)] + [c for c in itertools.product((-1, 0, 1), repeat=3) if 1 <= sum(map(abs, c)) <= 2]
Q = len(C)
W = [1.0 / 3.0] + [1.0 / 18.0 if sum(map(abs, c)) == 1 else 1.0 / 36.0 for c in C[1:]]
BACK = [C.index(tuple(-a for a in c)) for c in C]


def _double_dot(A, c):
    """A:(c c - I/3) for a symmetric 3x3 tensor A (nested lists)."""
    return sum(A[a][b] * (c[a] * c[b] - (1.0 / 3.0 if a == b else 0.0)) for a in range(3) for b in range(3))


def _equilibrium_deviation(i, drho, j, P):
    """f_eq,i(1 + drho, j, P) - f_eq,i(1, 0, 0) from eq:fieq:
    w_i (rho + c.j/c_s^2 + (P - rho c_s^2 I):(c c - c_s^2 I)/(2 c_s^4))."""
    c = C[i]
    iso = -drho / 3.0                                   # the change of -rho c_s^2 I
    A = [[P[a][b] + (iso if a == b else 0.0) for b in range(3)] for a in range(3)]
    return W[i] * (drho + 3.0 * sum(c[a] * j[a] for a in range(3)) + 4.5 * _double_dot(A, c))


def step_operator(H, ky, kz, lam, mu, tau, q, order):
    """The matrix (19H x 19H, complex) of one step acting on the amplitudes
    f[i, x] (index i*H + x) of a disturbance exp(i (ky y + kz z)); lam, mu
    in lattice units (mu = 1/3)."""
    n = Q * H
    basis = np.eye(n, dtype=complex)
    f = {(i, x): basis[i * H + x] for i in range(Q) for x in range(H)}
    # value at (y, z) + (c_y, c_z) relative to (y, z)
    shift = [cmath.exp(1j * (ky * c[1] + kz * c[2])) for c in C]
    inside = lambda x: 0 <= x < H                                          # noqa: E731

    rho, j, P = {}, {}, {}
    for x in range(H):
        rho[x] = sum(f[(i, x)] for i in range(Q))
        j[x] = [sum(C[i][a] * f[(i, x)] for i in range(Q)) for a in range(3)]
        P[x] = [[sum(C[i][a] * C[i][b] * f[(i, x)] for i in range(Q)) for b in range(3)] for a in range(3)]

    def rho_across(x, i):
        xx = x + C[i][0]
        if inside(xx):
            return rho[xx] * shift[i]
        xb = x - C[i][0]
        if inside(xb):
            return 2.0 * rho[x] - rho[xb] * shift[BACK[i]]
        return rho[x]

    fcol = {}
    for x in range(H):
        g = [3.0 * sum(W[i] * C[i][a] * rho_across(x, i) for i in range(1, Q)) for a in range(3)]
        S = [(mu - lam) * g[a] for a in range(3)]
        u = [j[x][a] + 0.5 * S[a] for a in range(3)]
        for i in range(Q):
            feq = _equilibrium_deviation(i, rho[x], u, P[x])
            psi = 3.0 * W[i] * sum(C[i][a] * S[a] for a in range(3))
            fcol[(i, x)] = f[(i, x)] - (f[(i, x)] - feq) / tau + (1.0 - 0.5 / tau) * psi

    # Cauchy stress of a plane: sigma = -P - (lambda - mu) drho I
    sigma = {x: [[-P[x][a][b] - ((lam - mu) * rho[x] if a == b else 0.0) for b in range(3)] for a in range(3)]
             for x in range(H)}
    kappa = (1.0 - 2.0 * q) / (1.0 + 2.0 * q)
    beta = 2.0 / (1.0 + 2.0 * q)
    new = {}
    for x in range(H):
        for i in range(Q):
            src = x - C[i][0]
            if inside(src):
                new[(i, x)] = fcol[(i, src)] * shift[BACK[i]]
                continue
            # the link (x, k), k = BACK[i], leaves the slab through a wall
            kk = BACK[i]
            xin = x - C[kk][0]                          # plane of x - c_k
            thin = not inside(xin)
            back = shift[BACK[kk]]                      # x - c_k lies at (y, z) offset -c_k
            if order == 1 and not thin:
                drho_bd = (1.0 + q) * rho[x] - q * rho[xin] * back
                sb = [[(1.0 + q) * sigma[x][a][b] - q * sigma[xin][a][b] * back for b in range(3)]
                      for a in range(3)]
            else:
                drho_bd = rho[x]
                sb = sigma[x]
            # Pi = I - n n with n along x: the tangential (y, z) block of sigma_b
            star = [[sb[a][b] if (a > 0 and b > 0) else 0.0 * sb[a][b] for b in range(3)] for a in range(3)]
            Pstar = [[-star[a][b] - ((lam - mu) * drho_bd if a == b else 0.0) for b in range(3)] for a in range(3)]
            E = 2.0 * _equilibrium_deviation(kk, drho_bd, [0.0, 0.0, 0.0], Pstar)
            if thin:
                new[(i, x)] = -fcol[(kk, x)] + E
            else:
                new[(i, x)] = -fcol[(kk, x)] - kappa * (fcol[(kk, xin)] * back + fcol[(i, x)]) + beta * E
    A = np.zeros((n, n), dtype=complex)
    for (i, x), v in new.items():
        A[i * H + x] = v
    return A


def max_growth(H, ny, nz, lam_over_mu, tau, q, order):
    """Largest eigenvalue modulus of the one-step map over the wave vectors
    (2 pi a / ny, 2 pi b / nz) of a slab ny x nz sites wide (by symmetry,
    0 <= a <= ny/2 and 0 <= b < nz suffice)."""
    mu = 1.0 / 3.0
    lam = lam_over_mu * mu
    worst = 0.0
    for a in range(ny // 2 + 1):
        for b in range(nz):
            A = step_operator(H, 2.0 * math.pi * a / ny, 2.0 * math.pi * b / nz, lam, mu, tau, q, order)
            worst = max(worst, float(np.abs(np.linalg.eigvals(A)).max()))
    return worst
